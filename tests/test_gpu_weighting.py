"""Per-constraint gradient statistics on the GPU (pcls_constraint_grad_stats)
against the oracle, and one adaptive reweighting round."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import native as N  # noqa: E402
from paper_2606_06656_amd import pcls, synth  # noqa: E402
from paper_2606_06656_amd.weighting import adaptive_weights, gradient_magnitudes, reweight  # noqa: E402
from gpu_util import corner_mix, log, oracle_for, rows_of  # noqa: E402


@pytest.mark.parametrize("kmax,seed", [(8, 0), (64, 1), (256, 2)])
def test_grad_stats_match_oracle(kmax, seed):
    inst = synth.mixed_small(n=300, seed=seed, kmax=kmax, count=250)
    inst.weight = np.random.default_rng(seed).uniform(0.5, 2.0, inst.m).astype(np.float32)
    log(f"case grad stats kmax={kmax} m={inst.m}")
    prob = pcls.Problem.from_instance(inst)
    R = 37
    X = prob.state_from_rows(corner_mix(np.random.default_rng(seed), R, inst.n))
    got = prob.constraint_grad_stats(X, R).cpu().numpy().astype(np.float64)
    want = oracle_for(inst).constraint_grad_sq(rows_of(X, R))
    k = np.diff(inst.row_ptr)
    # FP32 terms (relative 1e-5 of each |dFE/dy| <= 1) and the 2^-s quantum
    tol = 2e-5 * np.sqrt(np.maximum(want, 0) * R * k) + 1e-5 * want + R * k * 2.0 ** -30
    assert np.all(np.abs(got - want) <= tol), np.max(np.abs(got - want) - tol)
    # repeatable bit for bit
    assert np.array_equal(prob.constraint_grad_stats(X, R).cpu().numpy(), got.astype(np.float32))


def test_grad_stats_errors_and_constants():
    inst = synth.Instance(n=3, row_ptr=np.array([0, 2, 3], np.int32), lit=np.array([1, -2, 3], np.int32),
                          ctype=np.array([2, 0], np.int8), param=np.array([0, 0], np.int32))  # CARD>=0 is constant
    prob = pcls.Problem.from_instance(inst)
    X = prob.state_from_rows(np.array([[0.2, -0.4, 0.9], [0.1, 0.1, -0.3]], np.float32))
    out = prob.constraint_grad_stats(X, 2).cpu().numpy()
    assert out[0] == 0.0 and out[1] == pytest.approx(2.0)  # OR of one literal: dFE/dy = 1 everywhere
    L = pcls.load_library()
    acc = torch.empty(2, dtype=torch.int64, device=prob.device)
    assert L.pcls_constraint_grad_stats(prob.handle, 0, pcls._tptr(X), pcls._tptr(acc), pcls._tptr(acc),
                                        pcls._stream()) == pcls.PCLS_E_INVALID


def test_reweighting_round_on_redundant_encoding():
    """EO written redundantly as CARD>=k-1 over the negated literals plus OR
    (the paper's redundant-encoding case): from restarts near the all-true
    corner, where the redundant pair is flat, one round raises the weights of
    the flattest constraints and keeps the mean weight; the reweighted problem
    evaluates against the oracle with its new weights."""
    k, reps = 6, 40
    rng = np.random.default_rng(5)
    n = 60
    rows, lits, types, params = [0], [], [], []
    for _ in range(reps):
        vs = rng.choice(n, k, replace=False) + 1
        lits += list(-vs)
        types.append(2)  # CARD >= k-1 of the negated literals
        params.append(k - 1)
        rows.append(len(lits))
        lits += list(vs)
        types.append(0)  # OR
        params.append(0)
        rows.append(len(lits))
    inst = synth.Instance(n=n, row_ptr=np.array(rows, np.int32), lit=np.array(lits, np.int32),
                          ctype=np.array(types, np.int8), param=np.array(params, np.int32))
    log("case reweight")
    prob = pcls.Problem.from_instance(inst)
    R = 64
    x = np.clip(-0.95 + 0.05 * rng.standard_normal((R, n)), -1, 1).astype(np.float32)
    X = prob.state_from_rows(x)
    mag = gradient_magnitudes(prob, X, R)
    w, prob2 = reweight(inst, prob, X, R, alpha=0.5)
    assert abs(w.mean() - 1.0) < 1e-5
    np.testing.assert_allclose(w, adaptive_weights(mag, alpha=0.5), rtol=1e-6)
    order = np.argsort(mag)
    assert w[order[0]] >= w[order[-1]]
    inst2 = synth.Instance(n=n, row_ptr=inst.row_ptr, lit=inst.lit, ctype=inst.ctype, param=inst.param, weight=w)
    obj, _ = prob2.evaluate(X, R)
    ref = oracle_for(inst2).evaluate(rows_of(X, R), method=N.PMF, want_grad=False)
    assert np.all(np.abs(obj.cpu().numpy() - ref["obj"]) <= 1e-5 * np.abs(w).sum())
