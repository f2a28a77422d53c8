"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same seeded inputs and compare them."""
from __future__ import annotations

import sys

import numpy as np

from oracle import native as N

TOL = 1e-5  # relative agreement asked of FP32 objective and gradient


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_for(inst, with_coefficients=True):
    return N.OracleProblem(inst.n, inst.row_ptr, inst.lit, inst.ctype, inst.param, inst.weight,
                           with_coefficients=with_coefficients)


def rows_of(X, R):
    """(n, R_pad) device state -> (R, n) float64 host rows (exact promotion)."""
    return X[:, :R].T.contiguous().cpu().numpy().astype(np.float64)


def range_scales(inst):
    """Range scale of each computed sum: |FE_c| <= 1 and |dFE_c/dy_i| <= 1, so the
    objective's terms are bounded by sum_c |w_c| and variable v's gradient terms by
    the weighted number of occurrences of v."""
    w = np.ones(inst.m) if inst.weight is None else np.abs(np.asarray(inst.weight, np.float64))
    vars_ = np.abs(inst.lit) - 1
    occ = np.repeat(w, np.diff(inst.row_ptr))
    sg = np.bincount(vars_, weights=occ, minlength=inst.n)
    return float(w.sum()), sg


def quantum_floor(inst, prob, R):
    """Absolute floor of the fixed-point gradient accumulator: every term is
    rounded to a multiple of 2^-S, so a variable's sum may differ from the exact
    sum of its FP32 terms by (number of terms) * 2^-(S+1)."""
    S = prob.launch_info(R)["grad_scale_log2"]
    occ = np.bincount(np.abs(inst.lit) - 1, minlength=inst.n).astype(np.float64)
    return occ * 2.0 ** -(S + 1)


def assert_obj_grad(obj_gpu, grad_rows_gpu, ref, tol=TOL, what="", inst=None, floor_g=None):
    """Mixed bound |dF| <= tol max(|F|, s_F), |dg| <= tol max(|g|, s_g) elementwise.

    With inst=None the scales are the oracle's sums of term magnitudes
    (value-relative: sum_c |w_c FE_c|, sum |w_c dFE_c/dy_i|); with inst given
    they are the range scales of `range_scales` (each term relative to its
    range [-1, 1], the reading used where a term is a cancelling sum over
    DFT nodes and may be zero while FP32 leaves a residue near 1e-7).
    floor_g adds the accumulator quantum (`quantum_floor`) to the gradient bound."""
    F = ref["obj"]
    if inst is None:
        sF, sg = ref["sig_obj"], ref["sig_grad"]
    else:
        sF, sgv = range_scales(inst)
        sF = np.full_like(F, sF)
        sg = None if ref["grad"] is None else np.broadcast_to(sgv, ref["grad"].shape)
    bound = tol * np.maximum(np.abs(F), sF) + 1e-30
    err = np.abs(obj_gpu.astype(np.float64) - F)
    worst = int(np.argmax(err / bound))
    assert np.all(err <= bound), (f"{what}: objective off at restart {worst}: gpu {obj_gpu[worst]!r} oracle "
                                  f"{F[worst]!r} bound {bound[worst]:.3g}")
    if grad_rows_gpu is not None:
        g = ref["grad"]
        gb = tol * np.maximum(np.abs(g), sg) + 1e-30
        if floor_g is not None:
            gb = gb + floor_g
        ge = np.abs(grad_rows_gpu.astype(np.float64) - g)
        if not np.all(ge <= gb):
            r, v = np.unravel_index(int(np.argmax(ge / gb)), ge.shape)
            raise AssertionError(f"{what}: gradient off at restart {r} var {v}: gpu {grad_rows_gpu[r, v]!r} "
                                 f"oracle {g[r, v]!r} bound {gb[r, v]:.3g}")
    return float(np.max(err / bound))


def corner_mix(rng, R, n):
    """Mixed evaluation points: uniform interior, near-corner, exact corners, zeros."""
    x = rng.uniform(-1, 1, (R, n))
    q = R // 4
    x[q:2 * q] = np.sign(x[q:2 * q]) * rng.uniform(0.9, 1.0, (q, n))
    x[2 * q:2 * q + q // 2] = np.where(rng.random((q // 2, n)) < 0.5, -1.0, 1.0)
    x[-1] = 0.0
    return x.astype(np.float32)
