"""Length-bucket tables and the autotuners.

A plan's bucket table decides which padded lengths its segments use, and with
them how the long constraints' literals are split over lane groups; each
per-literal term is a float32 product whose rounding depends on that split, so
two tables step iterates that agree to float32 rounding, each checked against
the oracle.  For a given table the gradient sums are exact fixed point, so the
tile and block sizes the autotuners pick leave the iterates bitwise unchanged."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import native as N  # noqa: E402
from paper_2606_06656_amd import autotune, pcls, synth  # noqa: E402
from paper_2606_06656_amd.batch import Batch  # noqa: E402
from gpu_util import assert_obj_grad, log, oracle_for, rows_of  # noqa: E402


def test_tables_step_identical_iterates_and_match_oracle():
    inst = synth.mixed_small(n=300, seed=41, kmax=64, count=700)
    R, lr = 96, 0.1
    out = {}
    for table in (0, 1):
        prob = pcls.Problem.from_instance(inst, bucket_table=table)
        log(f"case table {table}: segments {prob.info().n_segments}")
        X = prob.new_state(R)
        prob.init_restarts(X, R, 5)
        prob.step(X, R, lr, 6)
        obj, grad = prob.evaluate(X, R)
        ref = oracle_for(inst).evaluate(rows_of(X, R), method=N.PMF)
        assert_obj_grad(obj.cpu().numpy(), grad[:, :R].T.cpu().numpy(), ref, what=f"table {table}", inst=inst)
        out[table] = X[:, :R].clone()
    # same trajectory up to float32 rounding of the terms (6 steps of lr 0.1)
    assert float((out[0] - out[1]).abs().max()) < 1e-4


def test_tune_problem_record_cache_and_bitwise_steps(tmp_path):
    inst = synth.c2_mixed(seed=9, n=600, n_or=1800, n_xor=180, n_card=60)
    R, lr = 256, 0.1
    cache = os.path.join(str(tmp_path), "tune.json")
    rec = autotune.tune_problem(inst, R, lr, probe_steps=2, cache_path=cache)
    log(f"case tune problem: {rec}")
    assert rec["bucket_table"] in (0, 1) and rec["block_threads"] in (512, 1024) and not rec["cached"]
    assert rec["ms_per_step"] == min(c["ms_per_step"] for c in rec["candidates"])
    with open(cache) as f:
        assert len(json.load(f)) == 1
    assert autotune.tune_problem(inst, R, lr, cache_path=cache)["cached"]
    tuned = autotune.tuned_problem(inst, R, rec)
    assert tuned.launch_info(R)["tile_restarts"] == rec["tile_restarts"]
    assert tuned.info().bucket_table == rec["bucket_table"]
    base = pcls.Problem.from_instance(inst, bucket_table=rec["bucket_table"])  # the planner's default launch
    X, Y = tuned.new_state(R), base.new_state(R)
    tuned.init_restarts(X, R, 3)
    base.init_restarts(Y, R, 3)
    tuned.step(X, R, lr, 5)
    base.step(Y, R, lr, 5)
    assert torch.equal(X[:, :R], Y[:, :R])


def test_tune_batch_and_bitwise_equal_to_per_instance(tmp_path):
    """The batch under the table and configuration tune_batch picks is bitwise
    equal to per-instance launches of the same plans."""
    rng = np.random.default_rng(3)
    insts = [synth.mixed_small(n=int(rng.integers(80, 600)), seed=60 + i, kmax=40, count=400) for i in range(6)]
    Rs = [64, 33, 64, 100, 1, 64]
    rec = autotune.tune_batch(insts, Rs, 0.1, probe_steps=2, cache_path=os.path.join(str(tmp_path), "b.json"))
    log(f"case tune batch: {rec}")
    assert rec["bucket_table"] in (0, 1) and len(rec["per_table"]) == 2
    # one accumulator width on both sides (the batch uses one width per launch)
    probs = [pcls.Problem.from_instance(i, bucket_table=rec["bucket_table"], accumulator_bits=32) for i in insts]
    refs = [pcls.Problem.from_instance(i, bucket_table=rec["bucket_table"], accumulator_bits=32) for i in insts]
    states, ref_states = [], []
    for k, (p, q, R) in enumerate(zip(probs, refs, Rs)):
        X = p.new_state(R)
        p.init_restarts(X, R, 100 + k)
        states.append(X)
        ref_states.append(X.clone())
    b = Batch(probs, Rs, states)
    b.set_config(rec["block_threads"], rec["lds_budget"], 0, 32)
    b.step(0.1, 4)
    for q, R, Y in zip(refs, Rs, ref_states):
        q.step(Y, R, 0.1, 4)
    torch.cuda.synchronize()
    assert b.config()["accumulator_bits"] == 32
    for k, (X, Y, R) in enumerate(zip(states, ref_states, Rs)):
        assert refs[k].launch_info(R)["accumulator_bits"] == 32
        assert torch.equal(X[:, :R], Y[:, :R]), k
