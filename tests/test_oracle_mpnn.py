"""Pins of the FP64 reference network against facts outside itself:
central differences of its loss (the autograd gradient is not trusted on its
own), permutation equivariance, isolated variables, and the input features
against a direct count."""
import numpy as np
import pytest
import torch

from oracle import mpnn_ref as M
from paper_2606_06656_amd import synth


def as_tuple(inst):
    return (inst.n, inst.row_ptr, inst.lit, inst.ctype, inst.param)


def rand_flat(seed, scale=0.3):
    total = sum(int(np.prod(s)) for _, s in M.spec())
    return np.random.default_rng(seed).uniform(-scale, scale, total)


def test_gradient_matches_central_differences():
    inst = synth.mixed_small(n=9, seed=1, kmax=4, count=7)
    flat = rand_flat(1)
    y = np.random.default_rng(2).uniform(-1, 1, inst.n)
    loss, _, g = M.mse_and_grads([as_tuple(inst)], flat, [y])
    rng = np.random.default_rng(3)
    h = 1e-6
    for idx in rng.choice(len(flat), 40, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[idx] += h
        fm[idx] -= h
        lp = M.mse_and_grads([as_tuple(inst)], fp, [y])[0]
        lm = M.mse_and_grads([as_tuple(inst)], fm, [y])[0]
        assert (lp - lm) / (2 * h) == pytest.approx(g[idx], abs=1e-7, rel=1e-5)


def test_permutation_equivariance():
    inst = synth.random_ksat(12, 30, 3, seed=5)
    flat = rand_flat(6)
    x = M.forward([as_tuple(inst)], M.unflatten(flat)).detach().numpy()
    perm = np.random.default_rng(7).permutation(inst.n)  # new index of each variable
    lit = np.sign(inst.lit) * (perm[np.abs(inst.lit) - 1] + 1)
    cperm = np.random.default_rng(8).permutation(inst.m)
    rows = [lit[inst.row_ptr[c]:inst.row_ptr[c + 1]] for c in cperm]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])])
    inst2 = synth.Instance(inst.n, rp.astype(np.int32), np.concatenate(rows).astype(np.int32), inst.ctype[cperm],
                           inst.param[cperm])
    x2 = M.forward([as_tuple(inst2)], M.unflatten(flat)).detach().numpy()
    np.testing.assert_allclose(x2[perm], x, atol=1e-12)


def test_disjoint_union_is_per_instance():
    a = synth.random_ksat(10, 20, 3, seed=1)
    b = synth.mixed_small(n=14, seed=2, kmax=5, count=9)
    flat = rand_flat(9)
    xa = M.forward([as_tuple(a)], M.unflatten(flat)).detach().numpy()
    xb = M.forward([as_tuple(b)], M.unflatten(flat)).detach().numpy()
    xab = M.forward([as_tuple(a), as_tuple(b)], M.unflatten(flat)).detach().numpy()
    np.testing.assert_allclose(xab, np.concatenate([xa, xb]), atol=1e-12)


def test_features_count_occurrences():
    inst = synth.mixed_small(n=20, seed=4, kmax=6, count=15)
    fv, fc = M.features(*as_tuple(inst))
    var = np.abs(inst.lit) - 1
    np.testing.assert_allclose(fv[:, 0].numpy() * 8, np.bincount(var, minlength=inst.n))
    np.testing.assert_allclose(fv[:, 2].numpy() * 8, np.bincount(var[inst.lit < 0], minlength=inst.n))
    assert torch.all(fc[:, :7].sum(1) == 1)
    np.testing.assert_allclose(fc[:, 7].numpy() * 8, np.diff(inst.row_ptr))


def test_isolated_variable_gets_bias_path_only():
    # variable 3 occurs nowhere: its state depends only on its own features
    inst = synth.Instance(3, np.array([0, 2], np.int32), np.array([1, -2], np.int32), np.array([0], np.int8),
                          np.array([0], np.int32))
    flat = rand_flat(10)
    x1 = M.forward([as_tuple(inst)], M.unflatten(flat)).detach().numpy()
    inst2 = synth.Instance(3, np.array([0, 2], np.int32), np.array([-1, 2], np.int32), np.array([0], np.int8),
                           np.array([0], np.int32))
    x2 = M.forward([as_tuple(inst2)], M.unflatten(flat)).detach().numpy()
    assert x1[2] == pytest.approx(x2[2], abs=1e-15)
    assert abs(x1[0] - x2[0]) > 1e-6  # flipping signs changes the occurring variables
