"""Autotuners of the launch configuration, timed on real steps.

`tune_problem` chooses, for one problem and restart count, the length-bucket
table of the plan (every compiled length, or only the powers of two above 8),
the restarts per workgroup and the threads per workgroup of the resident
engine.  `tune_batch` chooses the bucket table of a batch of instances together
with the batched engine's configuration (threads per workgroup and LDS budget,
searched by the library's pcls_batch_autotune).  Both time short launches on
scratch states, never on the caller's, and cache the winner in a JSON file
keyed by a signature of the workload (sizes, the histogram of constraint
classes, the restart count and the device).

For one bucket table the gradients are exact fixed-point sums, so the tile and
block sizes change only the time, not the iterates; the table changes how long
constraints are split over lane groups and so the float32 rounding of their
terms (the iterates agree to that rounding).
"""
from __future__ import annotations

import hashlib
import json
import os
from collections import Counter

import numpy as np

from . import pcls

TABLES = (0, 1)  # pcls_plan_options.bucket_table


def _device_name(device) -> str:
    import torch
    return torch.cuda.get_device_name(torch.device(device))


def workload_signature(instances, restarts, device) -> str:
    """Sizes, class histogram ((type, length, parameter) counts), weights kind,
    restart counts and device of a workload."""
    h = hashlib.sha256()
    for inst, R in zip(instances, restarts):
        k = np.diff(inst.row_ptr)
        hist = Counter(zip(inst.ctype.tolist(), k.tolist(), inst.param.tolist()))
        w = "unit" if inst.weight is None or bool(np.all(inst.weight == 1)) else "weighted"
        h.update(f"{inst.n},{inst.m},{inst.L},{R},{w};".encode())
        h.update(repr(sorted(hist.items())).encode())
    h.update(_device_name(device).encode())
    return h.hexdigest()[:24]


def _load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store_cache(path, cache):
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)


def _time_steps(prob, R, lr, steps, reps=2):
    import torch
    X = prob.new_state(R)
    prob.init_restarts(X, R, 1)
    prob.step(X, R, lr, steps)  # warm-up launch of the same size
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        prob.step(X, R, lr, steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * steps)


def tune_problem(inst, R: int, lr: float = 0.1, probe_steps: int = 3, tables=TABLES, blocks=(1024, 512),
                 cache_path: str | None = None, device="cuda:0"):
    """Fastest (bucket table, restarts per workgroup, threads per workgroup) for
    R restarts of inst: the automatic tile, half and twice it, under each table
    and block size."""
    key = "problem:" + workload_signature([inst], [R], device)
    cache = _load_cache(cache_path)
    if key in cache:
        return dict(cache[key], cached=True)
    cands = []
    for table in tables:
        prob = pcls.Problem.from_instance(inst, device=device, bucket_table=table)
        T0 = prob.launch_info(R)["tile_restarts"]
        for T in sorted({max(1, T0 // 2), T0, min(64, 2 * T0)}):
            for block in blocks:
                try:
                    prob.set_launch(T, block)
                    ms = _time_steps(prob, R, lr, probe_steps)
                except pcls.PclsError:
                    continue  # tile does not fit or is too wide for the longest constraints
                cands.append({"bucket_table": table, "tile_restarts": T, "block_threads": block,
                              "ms_per_step": ms})
        prob.close()
    best = min(cands, key=lambda c: c["ms_per_step"])
    out = dict(best, probe_steps=probe_steps, candidates=cands, cached=False)
    cache[key] = out
    _store_cache(cache_path, cache)
    return out


def tuned_problem(inst, R: int, rec: dict, device="cuda:0") -> pcls.Problem:
    """The problem planned and launched as a tune_problem record says."""
    prob = pcls.Problem.from_instance(inst, device=device, bucket_table=rec["bucket_table"])
    prob.set_launch(rec["tile_restarts"], rec["block_threads"])
    return prob


def tune_batch(instances, restarts, lr: float = 0.1, probe_steps: int = 3, tables=TABLES,
               cache_path: str | None = None, device="cuda:0"):
    """Fastest (bucket table, batched-engine configuration) for a batch: under
    each table the instances are planned and the library's autotuner searches
    threads per workgroup x LDS budget on scratch states."""
    from .batch import Batch
    key = "batch:" + workload_signature(instances, restarts, device)
    cache = _load_cache(cache_path)
    if key in cache:
        return dict(cache[key], cached=True)
    per_table = []
    for table in tables:
        probs = [pcls.Problem.from_instance(i, device=device, bucket_table=table) for i in instances]
        states = []
        for k, (p, R) in enumerate(zip(probs, restarts)):
            X = p.new_state(R)
            p.init_restarts(X, R, k)
            states.append(X)
        b = Batch(probs, list(restarts), states)
        res = b.autotune(lr, probe_steps=probe_steps)
        per_table.append(dict(res, bucket_table=table))
        b.close()
        for p in probs:
            p.close()
    best = min(per_table, key=lambda r: r["probe_ms"])
    out = {"bucket_table": best["bucket_table"], "block_threads": best["block_threads"],
           "lds_budget": best["lds_budget"], "accumulator_bits": best["accumulator_bits"],
           "probe_ms": best["probe_ms"], "probe_steps": probe_steps,
           "per_table": [{k: r[k] for k in ("bucket_table", "block_threads", "lds_budget", "probe_ms")}
                         for r in per_table], "cached": False}
    cache[key] = out
    _store_cache(cache_path, cache)
    return out
