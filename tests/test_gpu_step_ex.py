"""pcls_step_ex: partial-assignment completion (fixed variables) and
convergence-aware stepping (per-restart iteration counts, early retirement)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import coeffs as C  # noqa: E402
from oracle import native as N  # noqa: E402
from paper_2606_06656_amd import pcls, synth  # noqa: E402
from gpu_util import TOL, log, oracle_for, range_scales, rows_of  # noqa: E402


def test_fixed_variables_hold_and_free_ones_follow_the_oracle():
    counts = {C.OR: 300, C.XOR: 20, C.CARD_GE: 30, C.NAE: 30}
    inst, z = synth.planted(150, counts, seed=3)
    log("case fixed variables")
    prob = pcls.Problem.from_instance(inst)
    rng = np.random.default_rng(3)
    fixed = np.zeros(inst.n, np.int8)
    sel = rng.choice(inst.n, int(0.2 * inst.n), replace=False)
    fixed[sel] = z[sel]
    fx = torch.tensor(fixed, device=prob.device)
    R, lr = 64, 0.1
    X = prob.new_state(R)
    prob.init_restarts(X, R, 5)
    for t in range(5):
        X0 = X.clone()
        prob.step_ex(X, R, lr, 1, fixed=fx)
        x0 = rows_of(X0, R)
        x0[:, sel] = z[sel]  # the kernel holds fixed variables before evaluating
        ref = oracle_for(inst).evaluate(x0, method=N.PMF)
        expect = np.clip(x0 - lr * ref["grad"], -1, 1)
        expect[:, sel] = z[sel]
        x1 = rows_of(X, R)
        slack = lr * TOL * np.maximum(np.abs(ref["grad"]), range_scales(inst)[1]) + 2.0 ** -22
        assert np.all(np.abs(x1 - expect) <= slack), t
        assert np.all(x1[:, sel] == z[sel])
    # longer run: the fixed 20% stay exactly at the planted values
    prob.step_ex(X, R, lr, 100, fixed=fx)
    assert np.all(rows_of(X, R)[:, sel] == z[sel])
    with pytest.raises(pcls.PclsError):
        prob.step_ex(X, R, lr, 1, fixed=torch.zeros(inst.n + 1, dtype=torch.int8, device=prob.device))


@pytest.mark.parametrize("T", [1, 4])
def test_convergence_counts_and_retirement(T):
    inst = synth.c1_3sat(7)
    log(f"case convergence T={T}")
    prob = pcls.Problem.from_instance(inst)
    prob.set_launch(T, 256)
    R, lr, S, tol = 64, 0.1, 150, 1e-4
    X = prob.new_state(R)
    prob.init_restarts(X, R, 9)
    ref = X.clone()
    tr, iters = prob.step_ex(X, R, lr, S, trace=True, tol=tol, want_iters=True)
    it = iters.cpu().numpy()
    # replay step by step (bitwise identical trajectories: exact gradient sums)
    first = np.full(R, S)
    traj = []
    for s in range(S):
        prev = ref.clone()
        prob.step(ref, R, lr, 1)
        traj.append(ref.clone())
        dx = (ref[:, :R] - prev[:, :R]).abs().max(dim=0).values.cpu().numpy()
        newly = (first == S) & (dx < tol)
        first[newly] = s + 1
    assert np.array_equal(it, first), (it, first)
    # a retired tile stops stepping: its restarts hold the state of the step at which
    # the last restart of the tile converged
    x_end = X[:, :R].cpu()
    for r0 in range(0, R, T):
        stop = int(first[r0:r0 + T].max())
        expect = traj[stop - 1][:, r0:r0 + T].cpu()
        assert torch.equal(x_end[:, r0:r0 + T], expect), r0
    # trace entries after retirement repeat the last evaluated objective
    trn = tr.cpu().numpy()
    for r in range(R):
        stop = int(first[(r // T) * T:(r // T) * T + T].max())
        if stop < S:
            assert np.all(trn[stop:, r] == trn[stop - 1, r]) or stop == 0
