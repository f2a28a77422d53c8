"""Adaptive constraint weighting from per-constraint gradient magnitudes.

The paper names this as the remedy for the plateaus that redundant or
symmetric encodings create (Case Studies, "Redundant Constraint Effect": at the
all-true corner the EO constraint's gradient is small and projected gradient
descent stalls; Conclusions, future work (i)) and fixes no scheme.  The reading
implemented here:

    g_c  = sqrt( mean over restarts of sum_i (dFE_c/dy_i)^2 )        (GPU kernel)
    w_c <- w_c * clip( (g_bar / max(g_c, eps g_bar))^alpha, lo, hi ),
    g_bar = mean of g_c over the non-constant constraints,

then rescaled so that the mean weight is unchanged.  Constraints whose relaxed
value is flat where the restarts sit (small g_c) gain weight, steep ones lose
it; alpha = 0 leaves the weights unchanged.  New weights enter through a
re-plan (the fixed-point scales depend on them).
"""
from __future__ import annotations

import numpy as np


def gradient_magnitudes(problem, X, R: int) -> np.ndarray:
    """RMS over the R restarts of each constraint's unweighted literal gradient
    (caller's constraint order), from pcls_constraint_grad_stats."""
    sq = problem.constraint_grad_stats(X, R).cpu().numpy().astype(np.float64)
    return np.sqrt(np.maximum(sq, 0.0) / R)


def adaptive_weights(mag, weights=None, alpha: float = 0.5, lo: float = 0.25, hi: float = 4.0,
                     eps: float = 1e-3, active=None) -> np.ndarray:
    """One reweighting round (see the module docstring).  `active` marks the
    constraints that take part (default: g_c > 0); the others keep their weight."""
    mag = np.asarray(mag, np.float64)
    w = np.ones_like(mag) if weights is None else np.asarray(weights, np.float64).copy()
    act = (mag > 0) if active is None else np.asarray(active, bool)
    if not act.any() or alpha == 0.0:
        return w.astype(np.float32)
    gbar = mag[act].mean()
    factor = (gbar / np.maximum(mag[act], eps * gbar)) ** alpha
    mean_before = w[act].mean()
    w[act] = w[act] * np.clip(factor, lo, hi)
    w[act] *= mean_before / w[act].mean()
    return w.astype(np.float32)


def reweight(inst, problem, X, R: int, alpha: float = 0.5, lo: float = 0.25, hi: float = 4.0, device=None):
    """Compute new weights for `inst` from the restarts X of `problem` and return
    (weights, new Problem planned with them)."""
    from . import pcls
    from .synth import Instance
    mag = gradient_magnitudes(problem, X, R)
    w0 = None if inst.weight is None else np.asarray(inst.weight, np.float64)
    w = adaptive_weights(mag, w0, alpha, lo, hi)
    new = Instance(n=inst.n, row_ptr=inst.row_ptr, lit=inst.lit, ctype=inst.ctype, param=inst.param, weight=w)
    return w, pcls.Problem.from_instance(new, device=device or problem.device)
