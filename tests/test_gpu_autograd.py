"""The FE objective as a torch.autograd.Function: backward against central
differences (exact for a multilinear objective up to rounding), against the FP64
oracle gradient, and against the library's own projected step."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import native as N  # noqa: E402
from paper_2606_06656_amd import pcls, synth  # noqa: E402
from paper_2606_06656_amd.autograd import FEObjective, fe_objective  # noqa: E402
from gpu_util import log, oracle_for, range_scales  # noqa: E402


def small_problem(seed=3):
    inst = synth.mixed_small(n=40, seed=seed, kmax=12, count=60)
    return inst, pcls.Problem.from_instance(inst)


@pytest.mark.parametrize("h", [0.5, 1e-2])
def test_backward_matches_central_differences(h):
    inst, prob = small_problem()
    log(f"case autograd fd h={h}")
    R = 8
    rng = np.random.default_rng(4)
    # points whose shifted copies x +- h stay inside the cube
    a = 1.0 - h
    x = torch.tensor(rng.uniform(-a, a, (R, inst.n)), dtype=torch.float32, device=prob.device,
                     requires_grad=True)
    F = fe_objective(prob, x)
    gF = torch.tensor(rng.uniform(0.5, 1.5, R), dtype=torch.float32, device=prob.device)
    (F * gF).sum().backward()
    gx = x.grad.cpu().numpy()
    # multilinear in each coordinate: the central difference is exact for any h
    xd = x.detach().cpu().numpy().astype(np.float64)
    op = oracle_for(inst)
    for v in range(inst.n):
        xp, xm = xd.copy(), xd.copy()
        xp[:, v] += h
        xm[:, v] -= h
        # the GPU evaluates the same polynomial at the shifted points
        Fp = fe_objective(prob, torch.tensor(xp, dtype=torch.float32, device=prob.device)).cpu().numpy()
        Fm = fe_objective(prob, torch.tensor(xm, dtype=torch.float32, device=prob.device)).cpu().numpy()
        fd = (Fp.astype(np.float64) - Fm) / (2 * h) * gF.cpu().numpy()
        # FP32 objective rounding ~ 1e-7 * sum|w| per evaluation, divided by 2h
        tol = 4e-7 * inst.m / h + 1e-5
        np.testing.assert_allclose(gx[:, v], fd, atol=tol)
        # exact FP64 central difference of the oracle equals the oracle gradient
        if v < 3:
            fo = (op.evaluate(xp, want_grad=False)["obj"] - op.evaluate(xm, want_grad=False)["obj"]) / (2 * h)
            ref = op.evaluate(xd)["grad"][:, v]
            np.testing.assert_allclose(fo, ref, atol=1e-9)


def test_backward_matches_oracle_gradient():
    inst, prob = small_problem(5)
    log("case autograd oracle")
    R = 33
    rng = np.random.default_rng(6)
    x = torch.tensor(rng.uniform(-1, 1, (R, inst.n)), dtype=torch.float32, device=prob.device, requires_grad=True)
    F = FEObjective.apply(x, prob)
    F.sum().backward()
    ref = oracle_for(inst).evaluate(x.detach().cpu().numpy().astype(np.float64), method=N.PMF)
    sF, sg = range_scales(inst)
    assert np.all(np.abs(F.detach().cpu().numpy() - ref["obj"]) <= 1e-5 * np.maximum(np.abs(ref["obj"]), sF))
    assert np.all(np.abs(x.grad.cpu().numpy() - ref["grad"]) <= 1e-5 * np.maximum(np.abs(ref["grad"]), sg))


def test_autograd_descent_equals_library_step():
    """x <- clip(x - lr * dF/dx) through torch equals pcls_step."""
    inst = synth.c1_3sat(4)
    prob = pcls.Problem.from_instance(inst)
    log("case autograd step")
    R, lr = 64, 0.1
    X = prob.new_state(R)
    prob.init_restarts(X, R, 4)
    x = X[:, :R].T.contiguous().clone().requires_grad_(True)
    F = fe_objective(prob, x)
    F.sum().backward()
    x_torch = torch.clamp(x.detach() - lr * x.grad, -1, 1)
    prob.step(X, R, lr, 1)
    assert torch.allclose(x_torch, X[:, :R].T, atol=2e-7, rtol=0)


def test_no_grad_path_and_shape_errors():
    inst, prob = small_problem(7)
    x = torch.zeros((5, inst.n), device=prob.device)
    with torch.no_grad():
        F = fe_objective(prob, x)
    assert F.shape == (5,)
    with pytest.raises(ValueError):
        fe_objective(prob, torch.zeros((5, inst.n + 1), device=prob.device))
    # outside the cube (or NaN) the fixed-point scales do not hold: refused, not evaluated
    for bad in (1.0 + 2.0 ** -20, -3.0, float("nan")):
        xb = torch.zeros((5, inst.n), device=prob.device)
        xb[2, 7] = bad
        with pytest.raises(ValueError):
            fe_objective(prob, xb)
    # the faces of the cube are inside
    F = fe_objective(prob, torch.ones((5, inst.n), device=prob.device))
    assert torch.isfinite(F).all()
