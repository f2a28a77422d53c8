"""Throughput benchmark of the FE objective + gradient + projected step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

A step is one pass of the whole hot path over the batch: for every restart and
every constraint, the literal gather, node products, objective, per-literal
gradient and scatter, then the projected step of every variable.  The default
workload is the mixed symmetric-PB instance (n = 2000 variables; 6000 random
3-clauses, 600 XOR-5 constraints with a random parity bit, 200 "at least 3 of 8"
cardinality constraints; 1024 restarts; float32 state), synthetic and seeded.

Metric: literal-evaluations per second, R * L * K / t, with t the device time
of K steps (inputs resident in HBM).  Printed as one JSON line with a roofline
object for the dominant kernel and the oracle's CPU rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FE obj+grad literal-evals/sec (% HBM roofline); learned vs random-init sat rate"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2606_06656_amd/csrc/pcls.hip", "paper_2606_06656_amd/csrc/plan.cpp",
                  "paper_2606_06656_amd/csrc/internal.h"]


def workload(name: str):
    from paper_2606_06656_amd import synth
    if name == "c2":
        return synth.c2_mixed(), 1024, 0.1, "mixed_pb_n2000_or3x6000_xor5x600_card3of8x200_R1024"
    if name == "c3":
        return synth.c3_long(), 4096, 0.1, "long_support_n20000_m40000_geomk3to256_R4096"
    if name == "c3long":
        return synth.c3_forced_long(), 512, 0.1, "forced_long_n20000_k64to256_R512"
    if name == "c4":
        return synth.c4_batch(256), 64, 0.1, "batch256_nlogu100to10000_or3r4.2_xor5r0.1_R64each"
    if name == "c1":
        return synth.c1_3sat(0), 64, 0.1, "3sat_n50_m213_R64"
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes_per_step(n: int, m: int, L: int, R: int) -> int:
    """4 B x gather + 4 B gradient contribution per literal-evaluation, state read
    and write per (variable, restart), constraint literal stream and row data."""
    return 8 * R * L + 8 * R * n + 4 * L + 8 * m


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# Instruction-issue roof of the vector ALUs: 256 CUs x 4 SIMDs, one wave64
# instruction per SIMD every 4 cycles, 2.4 GHz.
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4


def profile_record(kernel: str, workload_key: str, kind: str, steps_per_launch: int):
    """Per-launch figures ("traffic": HBM bytes from the FETCH_SIZE / WRITE_SIZE
    passes scaled by the copy calibration; "counters": SQ instruction counts)
    from a committed rocprofv3 run, if it was taken on the current kernel source
    with the same launch size; else None."""
    path = os.path.join(PROFILE_DIR, f"{kernel}_{workload_key}_{kind}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != kernel_source_hash() or rec.get("steps_per_launch") != steps_per_launch:
        return None
    return rec


def roofline(kernel: str, key: str, alg_bytes_per_launch: float, launch_ms: float, steps_per_launch: int):
    """Gather-model HBM roofline of the dominant kernel (algorithmic bytes per
    launch over the average launch time), with the measured HBM traffic and the
    binding on-chip resource when committed profiles of this kernel exist."""
    achieved = alg_bytes_per_launch / (launch_ms / 1e3) / 1e9
    tr = profile_record(kernel, key, "traffic", steps_per_launch)
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None if tr is None else tr["hbm_bytes_per_launch"],
           "kernel": kernel, "launch_ms": launch_ms, "steps_per_launch": steps_per_launch,
           "model": "gather model: 8 B per literal-eval + 8 B per (variable, restart) + CSR per step"}
    if tr is not None:
        # HBM rate the counters measured: the state stays in LDS, so it is far below achieved
        out["traffic_gbs"] = tr["hbm_bytes_per_launch"] / (launch_ms / 1e3) / 1e9
    ct = profile_record(kernel, key, "counters", steps_per_launch)
    if ct is not None:
        from paper_2606_06656_amd import pcls
        rate = ct["valu_insts_per_launch"] / (launch_ms / 1e3) / 1e9
        out["binding"] = {"bound": "alu", "resource": "VALU instruction issue", "achieved": rate,
                          "peak": VALU_PEAK_GINST, "peak_measured": pcls.valu_issue_rate() / 1e9,
                          "unit": "G wave64-instr/s", "frac": rate / VALU_PEAK_GINST,
                          "valu_insts_per_launch": ct["valu_insts_per_launch"]}
    return out


def cpu_baseline(inst, lr: float, budget_s: float = 12.0, R_sample: int = 16):
    """The FP64 oracle (single-threaded C) on a bounded sample of the same
    workload: R_sample restarts, as many whole steps as fit in about budget_s."""
    import numpy as np

    from oracle import native as N
    from paper_2606_06656_amd import synth  # noqa: F401

    op = N.OracleProblem(inst.n, inst.row_ptr, inst.lit, inst.ctype, inst.param, inst.weight)
    x = N.init_uniform(R_sample, inst.n, 12345)
    steps = 0
    t0 = time.perf_counter()
    while True:
        res = op.evaluate(x, method=N.AUTO, want_sigma=False)
        x = N.step(x, res["grad"], lr)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    rate = R_sample * inst.L * steps / el
    out = {"value": rate, "unit": "literal-evals/s", "cores": 1, "kind": "oracle",
           "sample": f"{R_sample} restarts x {steps} steps of the same instance, FP64, single thread, "
                     f"{el:.1f} s"}
    out["all_cores"] = cpu_baseline_all_cores(op, inst, lr, budget_s, R_sample)
    return out


def cpu_baseline_all_cores(op, inst, lr: float, budget_s: float, R_sample: int):
    """The same oracle on every host core the box gives one GPU (at most 16): one
    thread per core, each stepping its own R_sample restarts (the oracle's C code
    keeps no shared state and ctypes releases the interpreter lock)."""
    import threading

    import numpy as np

    from oracle import native as N

    P = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    done = [0] * P

    def work(i):
        x = N.init_uniform(R_sample, inst.n, 777 + i)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            res = op.evaluate(x, method=N.AUTO, want_sigma=False)
            x = N.step(x, res["grad"], lr)
            done[i] += 1

    t0 = time.perf_counter()
    ths = [threading.Thread(target=work, args=(i,)) for i in range(P)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    el = time.perf_counter() - t0
    steps = int(np.sum(done))
    return {"value": R_sample * inst.L * steps / el, "unit": "literal-evals/s", "cores": P, "kind": "oracle",
            "sample": f"{P} threads x {R_sample} restarts, {steps} steps in total, {el:.1f} s"}


def bench_batch(args, insts, R, lr, key):
    """Many uneven instances: one persistent launch per captured graph replay
    (configuration from the autotuner) against per-instance plain launches."""
    import torch

    from paper_2606_06656_amd import pcls
    from paper_2606_06656_amd.batch import Batch

    probs = [pcls.Problem.from_instance(i, device="cuda:0") for i in insts]
    states = []
    for k, p in enumerate(probs):
        X = p.new_state(R)
        p.init_restarts(X, R, 4000 + k)
        states.append(X)
    S = args.graph_steps
    # every step writes each restart's objective (obj + grad per step)
    traces = [torch.empty((S, R), dtype=torch.float32, device="cuda:0") for _ in probs]
    b = Batch(probs, [R] * len(probs), states, traces)
    tune = b.autotune(lr, probe_steps=3, cache_path=args.tune_cache)
    reps = max(1, args.steps // S)
    steps = reps * S
    b.capture(lr, S)
    for _ in range(max(1, args.warmup // S)):
        b.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    L_tot = sum(i.L for i in insts)
    n_tot = sum(i.n for i in insts)
    m_tot = sum(i.m for i in insts)
    value = R * L_tot * steps / (ms / 1e3)
    # per-instance plain launches: one pcls_step(1) per instance per step
    bs = args.baseline_steps
    e0.record(stream)
    for _ in range(bs):
        for p, X in zip(probs, states):
            p.step(X, R, lr, 1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    base_rate = R * L_tot * bs / (ms_b / 1e3)
    alg = sum(algorithmic_bytes_per_step(i.n, i.m, i.L, R) for i in insts) * S
    cfg = b.config()
    out = {
        "metric": METRIC, "value": value, "unit": "literal-evals/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": key, "instances": len(insts), "sum_n": n_tot, "sum_m": m_tot, "sum_L": L_tot,
                   "restarts_each": R, "lr": lr, "graph_steps": S, "autotune": tune, "batch": cfg},
        "per_instance_launches": {"value": base_rate, "unit": "literal-evals/s", "steps": bs,
                                  "ms_per_step": ms_b / bs, "launches_per_step": len(insts),
                                  "speedup_of_batched": value / base_rate},
        "roofline": roofline("batch_kernel", key, alg, ms / reps, S),
    }
    print(json.dumps(out), flush=True)


WEIGHTS = os.path.join(ROOT, "paper_2606_06656_amd", "weights", "mpnn_3sat.npz")


def learned_vs_random(count=16, n=200, budgets=(0, 10, 50), R=64):
    """Second half of the metric: satisfied-constraint fraction of learned versus
    uniform restarts at equal step budgets on held-out random 3-SAT (ratio 4.2),
    using the committed network weights; None if no weights are committed."""
    if not os.path.exists(WEIGHTS):
        return None
    from paper_2606_06656_amd import learned as LRN
    from paper_2606_06656_amd import synth
    P, meta = LRN.Params.load(WEIGHTS, "cuda:0")
    insts = [synth.c5_eval(n, i) for i in range(count)]
    lrn = LRN.sat_fraction_curves(insts, list(budgets), R=R, seed=20000, P=P, gamma=meta["gamma"],
                                  sigma=meta["sigma"])
    uni = LRN.sat_fraction_curves(insts, list(budgets), R=R, seed=20000, P=None)
    rows = []
    for bi, S in enumerate(budgets):
        d = lrn["mean"][:, bi] - uni["mean"][:, bi]
        m, lo, hi = LRN.paired_bootstrap_ci(d, seed=S)
        rows.append({"steps": S, "sat_rate_learned": float(lrn["mean"][:, bi].mean()),
                     "sat_rate_random": float(uni["mean"][:, bi].mean()), "gain": m, "gain_ci95": [lo, hi],
                     "best_of_R_learned": float(lrn["best"][:, bi].mean()),
                     "best_of_R_random": float(uni["best"][:, bi].mean())})
    return {"instances": count, "n": n, "ratio": 4.2, "restarts": R, "statistic": "mean over restarts",
            "budgets": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c3long", "c4"])
    ap.add_argument("--steps-per-launch", type=int, default=100,
                    help="steps per launch of the resident kernel (timed and warm-up launches alike)")
    ap.add_argument("--graph-steps", type=int, default=50, help="c4: steps captured per graph replay")
    ap.add_argument("--tune-cache", default=None, help="c4: autotuner cache file (reused when present)")
    ap.add_argument("--baseline-steps", type=int, default=10, help="c4: steps of per-instance plain launches")
    ap.add_argument("--tile", type=int, default=0, help="restarts per workgroup (0 = auto)")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0 = auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-random restart comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (scales the HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.rand(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 5}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (restarts are independent, "
              "so several GPUs would each run their own share with no per-step exchange).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_06656_amd import pcls

    inst, R, lr, key = workload(args.workload)
    if args.workload == "c4":
        return bench_batch(args, inst, R, lr, key)
    prob = pcls.Problem.from_instance(inst, device="cuda:0")
    if args.tile or args.block:
        prob.set_launch(args.tile, args.block)
    X = prob.new_state(R)
    prob.init_restarts(X, R, 2)
    stream = torch.cuda.current_stream()
    S = max(1, min(args.steps_per_launch, args.steps))
    n_launch = max(1, args.steps // S)
    steps = n_launch * S
    # every step writes each restart's objective at its iterate (obj + grad per step)
    trace = torch.empty((S, R), dtype=torch.float32, device="cuda:0")
    for _ in range((args.warmup + S - 1) // S):
        prob.step(X, R, lr, S, trace=trace)
    torch.cuda.synchronize()

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(n_launch):
        prob.step(X, R, lr, S, trace=trace)  # one launch of the resident kernel runs S steps
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    t = ms / 1e3

    value = R * inst.L * steps / t
    last_obj = trace[-1]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "literal-evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": key, "n": inst.n, "m": inst.m, "L": inst.L, "restarts": R, "lr": lr,
                   "launch": prob.launch_info(R)},
        "objective_last_step": {"min": float(last_obj.min()), "mean": float(last_obj.mean())},
        "roofline": roofline("tile_kernel", key, algorithmic_bytes_per_step(inst.n, inst.m, inst.L, R) * S,
                             ms / n_launch, S),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, lr, args.cpu_budget)
    if args.workload == "c2" and not args.no_learned:
        out["learned_init"] = learned_vs_random()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
