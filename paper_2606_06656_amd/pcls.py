"""Python binding of libpcls (ctypes).

Argument marshalling only: every step of the evaluation runs in the library's
gfx950 kernels.  PyTorch provides device memory and the current HIP stream.

State layout: X is a float32 device tensor of shape (n, R_pad), restart index
contiguous, R_pad = round_up(R, 64).  `X[:, :R].T` is the (R, n) user view.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcls.so")

PCLS_OK, PCLS_E_INVALID, PCLS_E_UNSUPPORTED, PCLS_E_DUPVAR, PCLS_E_WORKSPACE, PCLS_E_HIP = range(6)
STATUS_NAMES = {0: "PCLS_OK", 1: "PCLS_E_INVALID", 2: "PCLS_E_UNSUPPORTED", 3: "PCLS_E_DUPVAR",
                4: "PCLS_E_WORKSPACE", 5: "PCLS_E_HIP"}

# exported entry points (checked by the CPU test suite against include/pcls.h)
EXPORTS = ["pcls_plan", "pcls_plan_ex", "pcls_problem_info", "pcls_upload", "pcls_init_restarts",
           "pcls_init_restarts_masked",
           "pcls_evaluate", "pcls_step", "pcls_step_ex", "pcls_extract", "pcls_set_launch", "pcls_launch_info",
           "pcls_destroy", "pcls_last_error",
           "pcls_batch_create", "pcls_batch_bind", "pcls_batch_set_config", "pcls_batch_get_config",
           "pcls_batch_step", "pcls_batch_capture", "pcls_batch_replay", "pcls_batch_autotune",
           "pcls_batch_destroy", "pcls_constraint_grad_stats", "pcls_constraint_grad_stats_noalloc"]


class PclsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class PlanOptions(ctypes.Structure):
    _fields_ = [("force_generic", ctypes.c_int32), ("accumulator_bits", ctypes.c_int32),
                ("bucket_table", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class StepOptions(ctypes.Structure):
    _fields_ = [("d_fixed", ctypes.c_void_p), ("tol", ctypes.c_float), ("d_iters", ctypes.c_void_p),
                ("reserved", ctypes.c_int32 * 4)]


class Info(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("n_cons", ctypes.c_int32), ("n_lits", ctypes.c_int64),
                ("max_len", ctypes.c_int32), ("n_classes", ctypes.c_int32), ("n_segments", ctypes.c_int32),
                ("accumulator_bits", ctypes.c_int32), ("grad_scale_log2_64", ctypes.c_int32),
                ("grad_scale_log2_32", ctypes.c_int32), ("obj_scale_log2", ctypes.c_int32),
                ("tile_restarts", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t), ("lds_bytes_per_restart", ctypes.c_size_t),
                ("cons_by_kind", ctypes.c_int32 * 5), ("bucket_table", ctypes.c_int32)]

KIND_NAMES = ("prod1", "prod2", "dft", "pmf", "const")


_lib = None


def load_library():
    """Load libpcls.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_06656_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i32, u64, vp, sz = ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.c_void_p
    L.pcls_plan.restype = i32
    L.pcls_plan.argtypes = [i32, i32, vp, vp, vp, vp, vp, ctypes.POINTER(P), ctypes.POINTER(sz)]
    L.pcls_plan_ex.restype = i32
    L.pcls_plan_ex.argtypes = [i32, i32, vp, vp, vp, vp, vp, ctypes.POINTER(PlanOptions), ctypes.POINTER(P),
                               ctypes.POINTER(sz)]
    L.pcls_problem_info.restype = i32
    L.pcls_problem_info.argtypes = [P, ctypes.POINTER(Info)]
    L.pcls_upload.restype = i32
    L.pcls_upload.argtypes = [P, vp, sz, vp]
    L.pcls_init_restarts.restype = i32
    L.pcls_init_restarts.argtypes = [P, i32, u64, vp, vp]
    L.pcls_init_restarts_masked.restype = i32
    L.pcls_init_restarts_masked.argtypes = [P, i32, u64, vp, vp, vp]
    L.pcls_evaluate.restype = i32
    L.pcls_evaluate.argtypes = [P, i32, vp, vp, vp, vp]
    L.pcls_step.restype = i32
    L.pcls_step.argtypes = [P, i32, vp, ctypes.c_float, i32, vp, vp]
    L.pcls_step_ex.restype = i32
    L.pcls_step_ex.argtypes = [P, i32, vp, ctypes.c_float, i32, vp, ctypes.POINTER(StepOptions), vp]
    L.pcls_extract.restype = i32
    L.pcls_extract.argtypes = [P, i32, vp, vp, vp, vp, vp]
    L.pcls_set_launch.restype = i32
    L.pcls_set_launch.argtypes = [P, i32, i32]
    L.pcls_launch_info.restype = i32
    ip = ctypes.POINTER(i32)
    L.pcls_launch_info.argtypes = [P, i32, ip, ip, ip, ip, ctypes.POINTER(sz)]
    L.pcls_destroy.restype = i32
    L.pcls_destroy.argtypes = [P]
    L.pcls_last_error.restype = ctypes.c_char_p
    L.pcls_last_error.argtypes = []
    L.pcls_constraint_grad_stats.restype = i32
    L.pcls_constraint_grad_stats.argtypes = [P, i32, vp, vp, vp, vp]
    L.pcls_constraint_grad_stats_noalloc.restype = i32
    L.pcls_constraint_grad_stats_noalloc.argtypes = [P, i32, vp, vp, vp]
    _lib = L
    return L


def check(status: int):
    if status != PCLS_OK:
        msg = load_library().pcls_last_error()
        raise PclsError(status, msg.decode() if msg else "")


def round_up64(R: int) -> int:
    return (int(R) + 63) // 64 * 64


def _ptr(a):
    return None if a is None else a.ctypes.data


def _tptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Host-side plan of a formula (no device memory)."""

    def __init__(self, n, row_ptr, lit, ctype, param=None, weight=None, force_generic=False, accumulator_bits=0,
                 bucket_table=0):
        L = load_library()
        self.n = int(n)
        self._row_ptr = np.ascontiguousarray(row_ptr, np.int32)
        self._lit = np.ascontiguousarray(lit, np.int32)
        self._type = np.ascontiguousarray(ctype, np.int8)
        self._param = None if param is None else np.ascontiguousarray(param, np.int32)
        self._weight = None if weight is None else np.ascontiguousarray(weight, np.float32)
        self.m = len(self._row_ptr) - 1
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        opts = PlanOptions()
        opts.force_generic = 1 if force_generic else 0
        opts.accumulator_bits = int(accumulator_bits)
        opts.bucket_table = int(bucket_table)
        st = L.pcls_plan_ex(self.n, self.m, _ptr(self._row_ptr), _ptr(self._lit), _ptr(self._type),
                            _ptr(self._param), _ptr(self._weight), ctypes.byref(opts), ctypes.byref(h),
                            ctypes.byref(ws))
        check(st)
        self.handle = h
        self.workspace_bytes = ws.value

    @classmethod
    def from_instance(cls, inst, force_generic=False, accumulator_bits=0, bucket_table=0):
        return cls(inst.n, inst.row_ptr, inst.lit, inst.ctype, inst.param, inst.weight, force_generic,
                   accumulator_bits, bucket_table)

    def info(self) -> Info:
        info = Info()
        check(load_library().pcls_problem_info(self.handle, ctypes.byref(info)))
        return info

    def set_launch(self, tile_restarts=0, block_threads=0):
        check(load_library().pcls_set_launch(self.handle, int(tile_restarts), int(block_threads)))

    def launch_info(self, R: int) -> dict:
        """Launch the library will use for R restarts (queries the current device)."""
        v = [ctypes.c_int32() for _ in range(4)]
        lds = ctypes.c_size_t()
        check(load_library().pcls_launch_info(self.handle, int(R), *[ctypes.byref(a) for a in v],
                                              ctypes.byref(lds)))
        return {"tile_restarts": v[0].value, "block_threads": v[1].value, "accumulator_bits": v[2].value,
                "grad_scale_log2": v[3].value, "lds_bytes": lds.value}

    def close(self):
        if getattr(self, "handle", None):
            load_library().pcls_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem(Plan):
    """A plan bound to a device workspace (a torch uint8 tensor)."""

    def __init__(self, n, row_ptr, lit, ctype, param=None, weight=None, force_generic=False, device="cuda",
                 accumulator_bits=0, bucket_table=0):
        import torch
        super().__init__(n, row_ptr, lit, ctype, param, weight, force_generic, accumulator_bits, bucket_table)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(max(self.workspace_bytes, 256) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        check(load_library().pcls_upload(self.handle, ctypes.c_void_p(base + self._ws_off), self.workspace_bytes,
                                          _stream()))

    @classmethod
    def from_instance(cls, inst, force_generic=False, device="cuda", accumulator_bits=0, bucket_table=0):
        return cls(inst.n, inst.row_ptr, inst.lit, inst.ctype, inst.param, inst.weight, force_generic, device,
                   accumulator_bits, bucket_table)

    # ---- state
    def new_state(self, R: int):
        import torch
        return torch.zeros((self.n, round_up64(R)), dtype=torch.float32, device=self.device)

    def state_from_rows(self, x_rows):
        """(R, n) array or tensor -> (n, R_pad) device state."""
        import torch
        x = torch.as_tensor(np.asarray(x_rows, np.float32) if not isinstance(x_rows, torch.Tensor) else x_rows,
                            dtype=torch.float32)
        R = x.shape[0]
        X = self.new_state(R)
        X[:, :R] = x.to(self.device).T
        return X

    def _check_state(self, X, R):
        import torch
        if not isinstance(X, torch.Tensor) or X.dtype != torch.float32 or not X.is_contiguous():
            raise PclsError(PCLS_E_INVALID, "state must be a contiguous float32 tensor")
        if tuple(X.shape) != (self.n, round_up64(R)):
            raise PclsError(PCLS_E_INVALID, f"state shape {tuple(X.shape)} != {(self.n, round_up64(R))}")
        if X.device != self.device:
            raise PclsError(PCLS_E_INVALID, "state on another device")

    # ---- operations
    def init_restarts(self, X, R: int, seed: int):
        self._check_state(X, R)
        check(load_library().pcls_init_restarts(self.handle, int(R), int(seed) & (2 ** 64 - 1), _tptr(X),
                                                _stream()))
        return X

    def init_restarts_masked(self, X, R: int, seed: int, mask):
        """Redraw only the restarts r with mask[r] != 0 (uint8 or bool device
        tensor of R entries), as init_restarts(seed) would draw them."""
        import torch
        self._check_state(X, R)
        if mask.device != self.device or mask.numel() != R or mask.dtype not in (torch.uint8, torch.bool):
            raise PclsError(PCLS_E_INVALID, "mask must be a uint8 or bool tensor of R entries on the problem's device")
        m = mask.contiguous()
        check(load_library().pcls_init_restarts_masked(self.handle, int(R), int(seed) & (2 ** 64 - 1), _tptr(m),
                                                       _tptr(X), _stream()))
        return X

    def evaluate(self, X, R: int, want_grad: bool = True):
        import torch
        self._check_state(X, R)
        obj = torch.empty(R, dtype=torch.float32, device=self.device)
        grad = torch.empty_like(X) if want_grad else None
        check(load_library().pcls_evaluate(self.handle, int(R), _tptr(X), _tptr(obj), _tptr(grad), _stream()))
        return obj, grad

    def step(self, X, R: int, lr: float, n_steps: int = 1, trace=False):
        """n_steps projected-gradient steps; trace=True returns a new [n_steps][R]
        objective trace, a float32 device tensor of that shape is written in place."""
        import torch
        self._check_state(X, R)
        if isinstance(trace, torch.Tensor):
            if trace.dtype != torch.float32 or tuple(trace.shape) != (n_steps, R) or trace.device != self.device \
                    or not trace.is_contiguous():
                raise PclsError(PCLS_E_INVALID, "trace must be a contiguous float32 [n_steps][R] device tensor")
            tr = trace
        else:
            tr = torch.empty((n_steps, R), dtype=torch.float32, device=self.device) if trace else None
        check(load_library().pcls_step(self.handle, int(R), _tptr(X), float(lr), int(n_steps), _tptr(tr),
                                       _stream()))
        return tr

    def step_ex(self, X, R: int, lr: float, n_steps: int, trace: bool = False, fixed=None, tol: float = 0.0,
                want_iters: bool = False):
        """pcls_step_ex: fixed = int8 [n] device tensor (0 free, -1 True, +1 False) or None;
        tol > 0 enables per-restart convergence (returns iters [R] when want_iters)."""
        import torch
        self._check_state(X, R)
        tr = torch.empty((n_steps, R), dtype=torch.float32, device=self.device) if trace else None
        it = torch.empty(R, dtype=torch.int32, device=self.device) if want_iters else None
        if fixed is not None:
            if fixed.dtype != torch.int8 or fixed.numel() != self.n or fixed.device != self.device:
                raise PclsError(PCLS_E_INVALID, "fixed must be an int8 tensor of n entries on the problem's device")
        opt = StepOptions(None if fixed is None else fixed.data_ptr(), float(tol),
                          None if it is None else it.data_ptr())
        check(load_library().pcls_step_ex(self.handle, int(R), _tptr(X), float(lr), int(n_steps), _tptr(tr),
                                          ctypes.byref(opt), _stream()))
        return tr, it

    def constraint_grad_stats(self, X, R: int):
        """Per constraint (caller's order): sum over the R restarts of the squared
        unweighted gradient with respect to the constraint's literal values."""
        import torch
        self._check_state(X, R)
        m = self.info().n_cons
        acc = torch.empty(max(m, 1), dtype=torch.int64, device=self.device)
        out = torch.zeros(m, dtype=torch.float32, device=self.device)
        check(load_library().pcls_constraint_grad_stats(self.handle, int(R), _tptr(X), _tptr(acc), _tptr(out),
                                                        _stream()))
        return out

    def constraint_grad_stats_noalloc(self, X, R: int, out):
        """The same statistic into a caller-provided float32 [m] tensor, through
        the entry point that allocates nothing (the library's static scratch)."""
        self._check_state(X, R)
        check(load_library().pcls_constraint_grad_stats_noalloc(self.handle, int(R), _tptr(X), _tptr(out),
                                                                _stream()))
        return out

    def extract(self, X, R: int, want_assign: bool = True):
        import torch
        self._check_state(X, R)
        assign = torch.empty((R, self.n), dtype=torch.int8, device=self.device) if want_assign else None
        unsat = torch.empty(R, dtype=torch.int32, device=self.device)
        best = torch.empty(1, dtype=torch.int32, device=self.device)
        check(load_library().pcls_extract(self.handle, int(R), _tptr(X), _tptr(assign), _tptr(unsat), _tptr(best),
                                          _stream()))
        return assign, unsat, best


def solve(problem: Problem, R: int, steps: int, lr: float = 0.1, seed: int = 0):
    """Random restarts + projected gradient descent + extraction."""
    X = problem.new_state(R)
    problem.init_restarts(X, R, seed)
    problem.step(X, R, lr, steps)
    assign, unsat, best = problem.extract(X, R)
    return X, assign, unsat, best


def solve_recycling(problem: Problem, R: int, rounds: int, steps_per_round: int, lr: float = 0.1,
                    tol: float = 1e-4, seed: int = 0):
    """Convergence-aware restarts with recycling: each round runs up to
    steps_per_round steps with the per-restart convergence test, extracts every
    restart, and redraws the restarts that converged (seed + round) while the
    others continue from where they are.  Returns the best assignment seen
    (fewest violated constraints, first found), its count, and per-round
    telemetry: restarts converged, fewest violations, mean steps taken."""
    import numpy as np
    import torch
    X = problem.new_state(R)
    problem.init_restarts(X, R, seed)
    best_unsat, best_assign, rounds_out = None, None, []
    for k in range(rounds):
        _, iters = problem.step_ex(X, R, lr, steps_per_round, tol=tol, want_iters=True)
        assign, unsat, best = problem.extract(X, R)
        it = iters.cpu().numpy()
        u = unsat.cpu().numpy()
        b = int(best.cpu().numpy()[0])
        if best_unsat is None or int(u[b]) < best_unsat:
            best_unsat, best_assign = int(u[b]), assign[b].cpu().numpy().copy()
        converged = it < steps_per_round
        rounds_out.append({"round": k, "converged": int(converged.sum()), "min_unsat": int(u.min()),
                           "mean_steps": float(it.mean())})
        if best_unsat == 0:
            break
        if k + 1 < rounds and converged.any():
            mask = torch.from_numpy(converged.astype(np.uint8)).to(problem.device)
            problem.init_restarts_masked(X, R, seed + k + 1, mask)
    return {"assign": best_assign, "unsat": best_unsat, "rounds": rounds_out, "state": X}
