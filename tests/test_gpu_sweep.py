"""Seeded random sweep over instance shapes: every constraint type at lengths up
to 256, both bucket tables, ragged restart counts and random or corner-heavy
points.  Each case is checked against the FP64 oracle (objective and gradient)
and, over the tile widths the launch allows, for bitwise equal iterates and
gradients after three steps (the gradient sums are exact fixed point)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import native as N  # noqa: E402
from paper_2606_06656_amd import pcls, synth  # noqa: E402
from gpu_util import assert_obj_grad, corner_mix, log, oracle_for, rows_of  # noqa: E402

KMAX = [12, 16, 24, 32, 40, 48, 64, 96, 128, 256]


@pytest.mark.parametrize("case", range(40))
def test_random_shapes(case):
    rng = np.random.default_rng(7000 + case)
    kmax = KMAX[case % len(KMAX)]
    n = int(rng.integers(max(80, kmax + 8), 600))
    seed = int(rng.integers(1 << 30))
    inst = synth.mixed_small(n=n, seed=seed, kmax=kmax, count=int(rng.integers(50, 400)))
    table = case % 2
    R = int(rng.integers(1, 140))
    log(f"case {case}: kmax {kmax} n {n} m {inst.m} table {table} R {R} seed {seed}")
    prob = pcls.Problem.from_instance(inst, bucket_table=table)
    prng = np.random.default_rng(seed)
    x = corner_mix(prng, R, inst.n) if case % 3 else prng.uniform(-1, 1, (R, inst.n))
    X = prob.state_from_rows(x)
    obj, grad = prob.evaluate(X, R)
    ref = oracle_for(inst).evaluate(rows_of(X, R), method=N.PMF)
    assert_obj_grad(obj.cpu().numpy(), grad[:, :R].T.cpu().numpy(), ref, what=f"case {case}", inst=inst)
    base = None
    for T in (1, 2, 4, 8):
        try:
            prob.set_launch(T, 512)
        except pcls.PclsError:
            continue  # T times the widest lane group exceeds a wave
        Y = X.clone()
        prob.step(Y, R, 0.1, 3)
        _, g = prob.evaluate(Y, R)
        cur = (Y[:, :R].clone(), g[:, :R].clone())
        if base is None:
            base = cur
        else:
            assert torch.equal(base[0], cur[0]) and torch.equal(base[1], cur[1]), f"T={T}"
    assert base is not None
    prob.close()
