"""Batched persistent engine: many uneven instances in one launch, hipGraph
capture/replay and the autotuner, checked against per-instance launches.

Gradients accumulate in exact, order-independent fixed point, so every restart's
trajectory depends only on its own state: batched and per-instance runs must
agree bitwise on the states, whatever tiles and workgroup shapes each uses."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2606_06656_amd import pcls, synth  # noqa: E402
from paper_2606_06656_amd.batch import Batch  # noqa: E402
from gpu_util import TOL, assert_obj_grad, log, oracle_for, range_scales, rows_of  # noqa: E402
from oracle import native as N  # noqa: E402


def make_instances(count=10, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(30, 3000))
        if i % 3 == 0:
            inst = synth.random_ksat(n, int(4.2 * n), 3, seed=seed * 100 + i)
        elif i % 3 == 1:
            inst = synth.c2_mixed(seed=seed * 100 + i, n=n, n_or=3 * n, n_xor=n // 10, n_card=n // 20)
        else:
            inst = synth.mixed_small(n=max(n, 80), seed=seed * 100 + i, kmax=40, count=2 * n)
        out.append(inst)
    return out


def setup(count=10, seed=0, R_list=None, bits=64):
    """Instances with one accumulator width, so that per-instance launches and the
    batch (one width per launch) accumulate identically."""
    insts = make_instances(count, seed)
    probs = [pcls.Problem.from_instance(i, accumulator_bits=bits) for i in insts]
    R_list = R_list or [int(r) for r in np.random.default_rng(seed + 1).choice([1, 33, 64, 100, 128], count)]
    states = []
    for k, (p, R) in enumerate(zip(probs, R_list)):
        X = p.new_state(R)
        p.init_restarts(X, R, 1000 + k)
        states.append(X)
    return insts, probs, R_list, states


@pytest.mark.parametrize("bits", [32, 64])
def test_batch_equals_per_instance_bitwise(bits):
    insts, probs, Rs, states = setup(10, 0, bits=bits)
    log(f"case batch bits={bits} R={Rs} n={[i.n for i in insts]}")
    ref_states = [X.clone() for X in states]
    traces = [torch.zeros((4, R), device=X.device) for R, X in zip(Rs, states)]
    b = Batch(probs, Rs, states, traces)
    cfg = b.config()
    assert cfg["n_items"] >= len(probs) and cfg["grid"] >= 1 and cfg["accumulator_bits"] == bits
    b.step(0.1, 4)
    for p, R, X in zip(probs, Rs, ref_states):
        p.step(X, R, 0.1, 4)
    torch.cuda.synchronize()
    for k, (X, Y, R) in enumerate(zip(states, ref_states, Rs)):
        assert torch.equal(X[:, :R], Y[:, :R]), f"instance {k}"
    # the trace holds F at the iterates before each step
    for k in (0, 4, 9):
        p, R = probs[k], Rs[k]
        Z = p.new_state(R)
        p.init_restarts(Z, R, 1000 + k)
        for s in range(4):
            obj, _ = p.evaluate(Z, R, want_grad=False)
            np.testing.assert_allclose(traces[k][s].cpu().numpy(), obj.cpu().numpy(), rtol=1e-6, atol=1e-4)
            p.step(Z, R, 0.1, 1)


def test_batch_objective_matches_oracle():
    insts, probs, Rs, states = setup(5, 3, [64, 17, 100, 64, 1])
    log("case batch oracle")
    traces = [torch.zeros((1, R), device=X.device) for R, X in zip(Rs, states)]
    x0 = [rows_of(X, R) for X, R in zip(states, Rs)]
    b = Batch(probs, Rs, states, traces)
    b.step(0.1, 1)
    for k, inst in enumerate(insts):
        ref = oracle_for(inst).evaluate(x0[k], method=N.PMF, want_grad=False)
        sF = inst.m
        err = np.abs(traces[k][0].cpu().numpy() - ref["obj"])
        assert np.all(err <= 1e-5 * np.maximum(np.abs(ref["obj"]), sF)), k


def test_graph_capture_replay():
    insts, probs, Rs, states = setup(8, 5)
    log("case batch graph")
    eager = [X.clone() for X in states]
    b = Batch(probs, Rs, states)
    be = Batch(probs, Rs, eager)
    b.capture(0.1, 3)
    for rep in range(3):
        b.replay()
        be.step(0.1, 3)
        torch.cuda.synchronize()
        # eager work of the program between replays
        _ = [X.sum().item() for X in states]
        for k, (X, Y, R) in enumerate(zip(states, eager, Rs)):
            assert torch.equal(X[:, :R], Y[:, :R]), f"replay {rep} instance {k}"


def test_autotune_and_cache(tmp_path):
    insts, probs, Rs, states = setup(6, 7)
    log("case batch autotune")
    before = [X.clone() for X in states]
    b = Batch(probs, Rs, states)
    cache = os.path.join(str(tmp_path), "tune.json")
    res = b.autotune(0.1, probe_steps=2, cache_path=cache)
    assert res["block_threads"] in (256, 512, 1024) and not res["cached"]
    for X, Y, R in zip(states, before, Rs):
        assert torch.equal(X[:, :R], Y[:, :R])  # timing ran on scratch copies
    res2 = b.autotune(0.1, probe_steps=2, cache_path=cache)
    assert res2["cached"] and res2["block_threads"] == res["block_threads"]
    ref = [X.clone() for X in states]
    b.step(0.1, 2)
    for p, R, X in zip(probs, Rs, ref):
        p.step(X, R, 0.1, 2)
    for X, Y, R in zip(states, ref, Rs):
        assert torch.equal(X[:, :R], Y[:, :R])


@pytest.mark.parametrize("block,budget", [(256, 40 * 1024), (512, 80 * 1024), (1024, 0)])
def test_batch_configs_agree(block, budget):
    insts, probs, Rs, states = setup(6, 9, [64, 64, 33, 128, 5, 64])
    log(f"case batch config {block} {budget}")
    ref = [X.clone() for X in states]
    b = Batch(probs, Rs, states)
    try:
        b.set_config(block, budget)
    except pcls.PclsError as e:
        assert e.status == pcls.PCLS_E_UNSUPPORTED
        pytest.skip("an instance does not fit this LDS budget")
    b.step(0.05, 3)
    for p, R, X in zip(probs, Rs, ref):
        p.step(X, R, 0.05, 3)
    for X, Y, R in zip(states, ref, Rs):
        assert torch.equal(X[:, :R], Y[:, :R])


def test_batch_errors():
    insts, probs, Rs, states = setup(2, 11, [4, 4])
    b = Batch(probs, Rs, states)
    with pytest.raises(pcls.PclsError):
        b.set_config(block_threads=300)
    with pytest.raises(pcls.PclsError):
        b.replay()  # nothing captured
    with pytest.raises(pcls.PclsError):
        Batch(probs, [4, 0])


def test_short_traces_are_refused():
    """A bound trace receives n_steps rows per step: asking for more steps than
    it holds is refused before anything is launched."""
    insts, probs, Rs, states = setup(2, 13, [8, 8])
    traces = [torch.zeros((3, R), device=X.device) for R, X in zip(Rs, states)]
    b = Batch(probs, Rs, states, traces)
    b.step(0.1, 3)
    with pytest.raises(pcls.PclsError):
        b.step(0.1, 4)
    with pytest.raises(pcls.PclsError):
        b.capture(0.1, 5)


def test_c4_full_size_sampled():
    """256 uneven instances (n log-uniform on [100, 1e4], 64 restarts each) in one
    batched launch with the autotuned configuration, as bench.py times it: the
    objective of the first step and the first projected step of sampled
    (instance, restart) pairs against the oracle."""
    insts = synth.c4_batch(256)
    log(f"case c4 full size: sum n = {sum(i.n for i in insts)}")
    probs = [pcls.Problem.from_instance(i) for i in insts]
    R, lr = 64, 0.1
    states = []
    for k, p in enumerate(probs):
        X = p.new_state(R)
        p.init_restarts(X, R, 4000 + k)
        states.append(X)
    x0 = {k: rows_of(states[k], R) for k in (0, 77, 255)}
    traces = [torch.zeros((1, R), device=X.device) for X in states]
    b = Batch(probs, [R] * len(probs), states, traces)
    b.autotune(lr, probe_steps=2)
    b.capture(lr, 1)
    b.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for k, x in x0.items():
        rs = np.sort(rng.choice(R, 6, replace=False))
        ref = oracle_for(insts[k]).evaluate(x[rs], method=N.PMF)
        assert_obj_grad(traces[k][0].cpu().numpy()[rs], None, ref, what=f"c4 instance {k}", inst=insts[k])
        expect = np.clip(x[rs] - lr * ref["grad"], -1, 1)
        got = rows_of(states[k], R)[rs]
        slack = lr * TOL * np.maximum(np.abs(ref["grad"]), range_scales(insts[k])[1]) + 2.0 ** -22
        assert np.all(np.abs(got - expect) <= slack), k
