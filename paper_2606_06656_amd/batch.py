"""Batched execution of many instances (ctypes binding of the pcls_batch_* ABI)
and the autotuner's cache.

A `Batch` runs every instance's restarts in one persistent launch, optionally
replayed from a captured HIP graph.  `autotune` times the library's candidate
configurations on scratch copies of the states (the real states do not advance)
and caches the winner in a JSON file keyed by the batch's shape.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

from . import pcls


class BatchConfig(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("lds_budget", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("accumulator_bits", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_bound = False


def _lib():
    global _bound
    L = pcls.load_library()
    if not _bound:
        i32, vp, sz, f32 = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float
        L.pcls_batch_create.restype = i32
        L.pcls_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(vp),
                                        ctypes.POINTER(sz)]
        L.pcls_batch_bind.restype = i32
        L.pcls_batch_bind.argtypes = [vp, vp, sz, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.pcls_batch_set_config.restype = i32
        L.pcls_batch_set_config.argtypes = [vp, ctypes.POINTER(BatchConfig), vp]
        L.pcls_batch_get_config.restype = i32
        L.pcls_batch_get_config.argtypes = [vp, ctypes.POINTER(BatchConfig), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.pcls_batch_step.restype = i32
        L.pcls_batch_step.argtypes = [vp, f32, i32, vp]
        L.pcls_batch_capture.restype = i32
        L.pcls_batch_capture.argtypes = [vp, f32, i32, vp]
        L.pcls_batch_replay.restype = i32
        L.pcls_batch_replay.argtypes = [vp, vp]
        L.pcls_batch_autotune.restype = i32
        L.pcls_batch_autotune.argtypes = [vp, f32, i32, vp, ctypes.POINTER(BatchConfig), ctypes.POINTER(f32)]
        L.pcls_batch_destroy.restype = i32
        L.pcls_batch_destroy.argtypes = [vp]
        _bound = True
    return L


BATCH_EXPORTS = ["pcls_batch_create", "pcls_batch_bind", "pcls_batch_set_config", "pcls_batch_get_config",
                 "pcls_batch_step", "pcls_batch_capture", "pcls_batch_replay", "pcls_batch_autotune",
                 "pcls_batch_destroy"]


class Batch:
    """problems: list of pcls.Problem (uploaded); restarts: list of R_i."""

    def __init__(self, problems, restarts, states=None, traces=None):
        import torch
        L = _lib()
        self.problems = list(problems)
        self.restarts = [int(r) for r in restarts]
        n = len(self.problems)
        arr = (ctypes.c_void_p * n)(*[p.handle.value for p in self.problems])
        rs = (ctypes.c_int32 * n)(*self.restarts)
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        pcls.check(L.pcls_batch_create(arr, n, rs, ctypes.byref(h), ctypes.byref(ws)))
        self.handle = h
        self.workspace_bytes = ws.value
        dev = self.problems[0].device
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        self._ws = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        self.states = states if states is not None else [p.new_state(r) for p, r in zip(self.problems, self.restarts)]
        self.traces = traces
        self.bind(self.states, traces)

    def bind(self, states, traces=None):
        L = _lib()
        n = len(self.problems)
        for p, r, X in zip(self.problems, self.restarts, states):
            p._check_state(X, r)
        xs = (ctypes.c_void_p * n)(*[X.data_ptr() for X in states])
        if traces is not None:
            for i, (t, r) in enumerate(zip(traces, self.restarts)):
                if t is not None and (t.dtype.itemsize != 4 or t.dim() != 2 or t.shape[1] != r
                                      or t.device != states[i].device):
                    raise pcls.PclsError(pcls.PCLS_E_INVALID, f"trace {i} must be float32 [steps][{r}] on the device")
        tr = None if traces is None else (ctypes.c_void_p * n)(*[0 if t is None else t.data_ptr() for t in traces])
        pcls.check(L.pcls_batch_bind(self.handle, ctypes.c_void_p(self._ws), self.workspace_bytes, xs, tr,
                                     pcls._stream()))
        self.states, self.traces = list(states), traces

    def config(self):
        c = BatchConfig()
        n_items, grid = ctypes.c_int32(), ctypes.c_int32()
        pcls.check(_lib().pcls_batch_get_config(self.handle, ctypes.byref(c), ctypes.byref(n_items),
                                                ctypes.byref(grid)))
        d = c.as_dict()
        d.update(n_items=n_items.value, grid=grid.value)
        return d

    def set_config(self, block_threads=0, lds_budget=0, wgs_per_cu=0, accumulator_bits=0):
        c = BatchConfig(block_threads, lds_budget, wgs_per_cu, accumulator_bits)
        pcls.check(_lib().pcls_batch_set_config(self.handle, ctypes.byref(c), pcls._stream()))

    def _check_traces(self, n_steps: int):
        """Bound traces receive n_steps rows per step call: refuse shorter ones."""
        if self.traces is None:
            return
        for i, (t, r) in enumerate(zip(self.traces, self.restarts)):
            if t is None:
                continue
            if t.dim() != 2 or t.shape[0] < n_steps or t.shape[1] != r or not t.is_contiguous():
                raise pcls.PclsError(pcls.PCLS_E_INVALID,
                                     f"trace {i} must be a contiguous [>= {n_steps}][{r}] tensor, got {tuple(t.shape)}")

    def step(self, lr: float, n_steps: int):
        self._check_traces(n_steps)
        pcls.check(_lib().pcls_batch_step(self.handle, float(lr), int(n_steps), pcls._stream()))

    def capture(self, lr: float, n_steps: int):
        self._check_traces(n_steps)
        pcls.check(_lib().pcls_batch_capture(self.handle, float(lr), int(n_steps), pcls._stream()))

    def replay(self):
        pcls.check(_lib().pcls_batch_replay(self.handle, pcls._stream()))

    def signature(self) -> str:
        h = hashlib.sha256()
        for p, r in zip(self.problems, self.restarts):
            info = p.info()
            h.update(f"{info.n_vars},{info.n_cons},{info.n_lits},{info.max_len},{r};".encode())
        return h.hexdigest()[:20]

    def autotune(self, lr: float = 0.1, probe_steps: int = 5, cache_path: str | None = None):
        """Pick the fastest configuration (cached by signature); the bound states
        are swapped for scratch copies while timing, so they do not advance."""
        import torch
        key = self.signature()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key in cache:
            c = cache[key]
            self.set_config(c["block_threads"], c["lds_budget"], 0, c.get("accumulator_bits", 0))
            return dict(c, cached=True)
        real_states, real_traces = self.states, self.traces
        scratch = [X.clone() for X in real_states]
        self.bind(scratch, None)
        best = BatchConfig()
        ms = ctypes.c_float()
        pcls.check(_lib().pcls_batch_autotune(self.handle, float(lr), int(probe_steps), pcls._stream(),
                                              ctypes.byref(best), ctypes.byref(ms)))
        torch.cuda.synchronize()
        self.bind(real_states, real_traces)
        self.set_config(best.block_threads, best.lds_budget, 0, best.accumulator_bits)
        out = dict(best.as_dict(), probe_ms=ms.value, probe_steps=probe_steps, cached=False)
        if cache_path:
            cache[key] = out
            os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib().pcls_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
