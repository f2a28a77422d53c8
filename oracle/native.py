"""ctypes binding of the FP64 oracle library (fe_oracle.c).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It shares no code with the HIP path.

Arrays use the oracle's own layout: x and grad are [R][n] float64, one full
assignment per row.  Spectra and coefficients of constraint c sit at offset
row_ptr[c] + c of the concatenated tables (k_c + 1 entries each).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import coeffs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ESP, PMF, AUTO = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile fe_oracle.c with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.orc_fe_esp.restype = ctypes.c_double
        L.orc_fe_esp.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_grad_esp.restype = None
        L.orc_grad_esp.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_fe_pmf.restype = ctypes.c_double
        L.orc_fe_pmf.argtypes = [ctypes.c_int, dp, dp]
        L.orc_grad_pmf.restype = None
        L.orc_grad_pmf.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_eval_constraint.restype = ctypes.c_int
        L.orc_eval_constraint.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, dp, dp, dp]
        L.orc_eval_problem.restype = ctypes.c_long
        L.orc_eval_problem.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, dp, dp, ctypes.c_int, dp,
                                       dp, dp, dp, dp, ctypes.c_int]
        L.orc_constraint_grad_sq.restype = None
        L.orc_constraint_grad_sq.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, ctypes.c_int, dp, dp]
        L.orc_step.restype = None
        L.orc_step.argtypes = [ctypes.c_long, dp, dp, ctypes.c_double, dp]
        L.orc_extract.restype = None
        L.orc_extract.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, dp, ctypes.c_int, dp,
                                  ctypes.POINTER(ctypes.c_int8), ip, ip]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_init_uniform.restype = None
        L.orc_init_uniform.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, dp]
        _lib = L
    return _lib


def _p(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------ one constraint

def fe_esp(a, y, want_cond=False):
    a, y = _f64(a), _f64(y)
    cond = ctypes.c_double(0.0)
    v = lib().orc_fe_esp(len(y), _p(a), _p(y), ctypes.byref(cond) if want_cond else None)
    return (v, cond.value) if want_cond else v


def grad_esp(a, y):
    a, y = _f64(a), _f64(y)
    g = np.zeros(len(y))
    lib().orc_grad_esp(len(y), _p(a), _p(y), _p(g))
    return g


def fe_pmf(sp, y):
    sp, y = _f64(sp), _f64(y)
    return lib().orc_fe_pmf(len(y), _p(sp), _p(y))


def grad_pmf(sp, y):
    sp, y = _f64(sp), _f64(y)
    g = np.zeros(len(y))
    lib().orc_grad_pmf(len(y), _p(sp), _p(y), _p(g))
    return g


def eval_constraint(ctype, k, param, y, method=AUTO):
    """FE and per-literal gradient of one constraint at literal values y."""
    sp = coeffs.spectrum(ctype, k, param)
    a = _f64(coeffs.wf_coefficients_f64(sp))
    spa, y = _f64(sp), _f64(y)
    fe, cond = ctypes.c_double(), ctypes.c_double()
    g = np.zeros(k)
    used = lib().orc_eval_constraint(k, _p(spa), _p(a), _p(y), method, ctypes.byref(fe), _p(g),
                                     ctypes.byref(cond))
    return fe.value, g, used


# ------------------------------------------------------------ whole problem

class OracleProblem:
    """A CSR formula prepared for the oracle: spectra and exact coefficients."""

    def __init__(self, n, row_ptr, lit, ctype, param=None, weight=None, with_coefficients=True):
        self.n = int(n)
        self.row_ptr = _i32(row_ptr)
        self.lit = _i32(lit)
        self.m = len(self.row_ptr) - 1
        ctype = np.asarray(ctype)
        param = np.zeros(self.m, np.int64) if param is None else np.asarray(param)
        self.weight = None if weight is None else _f64(weight)
        total = int(self.row_ptr[-1]) + self.m
        self.sp_all = np.empty(total)
        self.coef_all = np.empty(total) if with_coefficients else None
        cache = {}
        for c in range(self.m):
            b, e = int(self.row_ptr[c]), int(self.row_ptr[c + 1])
            k = e - b
            key = (int(ctype[c]), k, int(param[c]))
            if key not in cache:
                sp = coeffs.spectrum(*key)
                cache[key] = (np.array(sp, np.float64),
                              np.array(coeffs.wf_coefficients_f64(sp)) if with_coefficients else None)
            sp, a = cache[key]
            self.sp_all[b + c:e + c + 1] = sp
            if with_coefficients:
                self.coef_all[b + c:e + c + 1] = a

    def evaluate(self, x, method=AUTO, want_grad=True, want_sigma=True):
        """x: [R][n] -> dict(obj[R], grad[R][n], sig_obj[R], sig_grad[R][n], n_pmf)."""
        x = _f64(np.atleast_2d(x))
        R = x.shape[0]
        assert x.shape[1] == self.n
        obj = np.zeros(R)
        grad = np.zeros((R, self.n)) if want_grad else None
        so = np.zeros(R) if want_sigma else None
        sg = np.zeros((R, self.n)) if (want_sigma and want_grad) else None
        coef = self.coef_all if method != PMF else None
        n_pmf = lib().orc_eval_problem(self.n, self.m, _p(self.row_ptr, ctypes.c_int32),
                                       _p(self.lit, ctypes.c_int32), _p(self.sp_all), _p(coef),
                                       _p(self.weight), R, _p(x), _p(obj), _p(grad), _p(so), _p(sg),
                                       method)
        return {"obj": obj, "grad": grad, "sig_obj": so, "sig_grad": sg, "n_pmf": int(n_pmf)}

    def constraint_grad_sq(self, x):
        """x: [R][n] -> [m]: per constraint, sum over rows of sum_i (dFE_c/dy_i)^2."""
        x = _f64(np.atleast_2d(x))
        out = np.zeros(self.m)
        lib().orc_constraint_grad_sq(self.n, self.m, _p(self.row_ptr, ctypes.c_int32), _p(self.lit, ctypes.c_int32),
                                     _p(self.sp_all), x.shape[0], _p(x), _p(out))
        return out

    def extract(self, x):
        x = _f64(np.atleast_2d(x))
        R = x.shape[0]
        assign = np.zeros((R, self.n), np.int8)
        unsat = np.zeros(R, np.int32)
        best = np.zeros(1, np.int32)
        lib().orc_extract(self.n, self.m, _p(self.row_ptr, ctypes.c_int32), _p(self.lit, ctypes.c_int32),
                          _p(self.sp_all), R, _p(x), _p(assign, ctypes.c_int8), _p(unsat, ctypes.c_int32),
                          _p(best, ctypes.c_int32))
        return assign, unsat, int(best[0])


def step(x, grad, lr):
    x, grad = _f64(x), _f64(grad)
    out = np.empty_like(x)
    lib().orc_step(x.size, _p(x), _p(grad), float(lr), _p(out))
    return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


def init_uniform(R, n, seed):
    x = np.zeros((R, n))
    lib().orc_init_uniform(int(R), int(n), ctypes.c_uint64(seed & (2 ** 64 - 1)), _p(x))
    return x
