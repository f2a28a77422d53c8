"""Train the learned restart initialiser and evaluate it against uniform restarts.

    python -m paper_2606_06656_amd.train_init --out paper_2606_06656_amd/weights/mpnn_3sat.npz \
        --report report.json

1. Training instances: random 3-SAT, n = 200, m = 840 (ratio 4.2), seeds 10000+i.
2. Labels: plain CLS (64 restarts, 500 projected-gradient steps, lr 0.1); the
   label of a variable is the mean corner value over the restarts with the
   fewest violated constraints.
3. Training: mean-squared error, Adam, the library's forward/backward kernels.
4. gamma and sigma of the proposal clip(gamma x_hat + sigma u) are chosen on
   held-out instances of the training distribution (seeds after the training set).
5. Evaluation on n in {200, 1000, 2000} at ratio 4.2 (seeds 20000+i, disjoint):
   satisfied-constraint fraction, best over restarts and mean over restarts, at
   equal step budgets, learned versus uniform initialisation, paired per
   instance, with bootstrap confidence intervals.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def select_proposal(P, instances, budgets=(0, 10, 50), grid_gamma=(0.5, 1.0, 2.0), grid_sigma=(0.25, 0.5, 1.0),
                    R=64, seed=7000):
    from . import learned as LRN
    best = None
    table = []
    for g in grid_gamma:
        for s in grid_sigma:
            res = LRN.sat_fraction_curves(instances, list(budgets), R=R, seed=seed, P=P, gamma=g, sigma=s)
            score = float(res["mean"].mean())
            table.append({"gamma": g, "sigma": s, "score": score})
            if best is None or score > best[2]:
                best = (g, s, score)
    return best[0], best[1], table


def evaluate(P, gamma, sigma, sizes=(200, 1000, 2000), count=32, budgets=(0, 10, 50, 200), R=64, seed=20000,
             log=print):
    from . import learned as LRN
    from . import synth
    out = {}
    for n in sizes:
        insts = [synth.c5_eval(n, i) for i in range(count)]
        lrn = LRN.sat_fraction_curves(insts, list(budgets), R=R, seed=seed, P=P, gamma=gamma, sigma=sigma)
        uni = LRN.sat_fraction_curves(insts, list(budgets), R=R, seed=seed, P=None)
        rows = []
        for bi, S in enumerate(budgets):
            row = {"steps": S}
            for kind in ("best", "mean"):
                d = lrn[kind][:, bi] - uni[kind][:, bi]
                m, lo, hi = LRN.paired_bootstrap_ci(d, seed=n + S)
                row[kind] = {"learned": float(lrn[kind][:, bi].mean()), "uniform": float(uni[kind][:, bi].mean()),
                             "gain": m, "ci95": [lo, hi]}
            rows.append(row)
            log(f"n={n} S={S}: mean-over-R learned {row['mean']['learned']:.4f} uniform "
                f"{row['mean']['uniform']:.4f} gain {row['mean']['gain']:+.4f} CI {row['mean']['ci95']}; "
                f"best-of-R gain {row['best']['gain']:+.4f}")
        out[str(n)] = {"instances": count, "restarts": R, "fallback_used": int(sum(not u for u in lrn["learned_used"])),
                       "budgets": rows}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--heldout", type=int, default=32)
    ap.add_argument("--label-steps", type=int, default=500)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-count", type=int, default=32)
    args = ap.parse_args()

    import torch

    from . import learned as LRN
    from . import synth
    log = lambda s: print(s, flush=True)  # noqa: E731
    t0 = time.time()
    train_set = [synth.c5_train(i) for i in range(args.train)]
    labels, best_unsat = LRN.cls_labels(train_set, restarts=64, steps=args.label_steps, seed=1)
    log(f"labels: {len(labels)} instances, mean best unsat {np.mean(best_unsat):.2f} "
        f"(solved {np.mean(np.array(best_unsat) == 0):.2%}) [{time.time() - t0:.1f}s]")
    P, hist = LRN.train(train_set, labels, steps=args.steps, batch_size=args.batch, lr=args.lr, log_every=100,
                        log=log)
    log(f"trained [{time.time() - t0:.1f}s]")
    held = [synth.c5_train(args.train + i) for i in range(args.heldout)]
    gamma, sigma, table = select_proposal(P, held)
    log(f"proposal gamma={gamma} sigma={sigma} [{time.time() - t0:.1f}s]")
    meta = {"train_instances": args.train, "label_steps": args.label_steps, "steps": args.steps,
            "batch": args.batch, "lr": args.lr, "gamma": gamma, "sigma": sigma, "loss_history": hist,
            "proposal_grid": table}
    P.save(args.out, meta)
    report = {"meta": meta, "evaluation": evaluate(P, gamma, sigma, count=args.eval_count, log=log),
              "seconds": time.time() - t0}
    torch.cuda.synchronize()
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    log(f"done [{time.time() - t0:.1f}s]")


if __name__ == "__main__":
    main()
