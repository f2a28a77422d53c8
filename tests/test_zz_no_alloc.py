"""pcls_constraint_grad_stats_noalloc, the entry point for callers that cannot
allocate device memory, against pcls_constraint_grad_stats (the same kernels
with a caller-owned accumulator): equal bit for bit on two calls in a row, the
second with a smaller problem and fewer restarts, so the static scratch is
reused with stale contents from the first call."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2606_06656_amd import pcls, synth  # noqa: E402
from gpu_util import corner_mix, log  # noqa: E402


def _stats_both(inst, R, seed):
    prob = pcls.Problem.from_instance(inst)
    X = prob.state_from_rows(corner_mix(np.random.default_rng(seed), R, inst.n))
    want = prob.constraint_grad_stats(X, R)
    got = torch.full((inst.m,), float("nan"), dtype=torch.float32, device=prob.device)
    L = pcls.load_library()
    pcls.check(L.pcls_constraint_grad_stats_noalloc(prob.handle, int(R), pcls._tptr(X), pcls._tptr(got),
                                                    pcls._stream()))
    torch.cuda.synchronize()
    return prob, X, want.cpu().numpy(), got.cpu().numpy()


def test_noalloc_stats_equal_allocating_entry_point():
    big = synth.mixed_small(n=400, seed=5, kmax=64, count=900)
    small = synth.mixed_small(n=90, seed=6, kmax=20, count=120)
    log(f"case noalloc big m={big.m} small m={small.m}")
    for inst, R, seed in ((big, 70, 1), (small, 9, 2)):
        _, _, want, got = _stats_both(inst, R, seed)
        assert np.all(np.isfinite(want)) and np.array_equal(got, want), (inst.m, R)
    # the second call on the smaller problem again after a larger one left its sums behind
    _, _, want, got = _stats_both(big, 33, 3)
    assert np.array_equal(got, want)


def test_noalloc_stats_limits_and_errors():
    inst = synth.mixed_small(n=50, seed=8, kmax=10, count=40)
    prob = pcls.Problem.from_instance(inst)
    X = prob.new_state(4)
    prob.init_restarts(X, 4, 1)
    out = torch.zeros(inst.m, dtype=torch.float32, device=prob.device)
    L = pcls.load_library()
    assert L.pcls_constraint_grad_stats_noalloc(prob.handle, 0, pcls._tptr(X), pcls._tptr(out),
                                                pcls._stream()) == pcls.PCLS_E_INVALID
    assert L.pcls_constraint_grad_stats_noalloc(prob.handle, 4, None, pcls._tptr(out),
                                                pcls._stream()) == pcls.PCLS_E_INVALID
    # more constraints than the static scratch holds: refused before any launch
    m = (1 << 18) + 1
    row_ptr = np.arange(m + 1, dtype=np.int32)
    lit = (np.arange(m, dtype=np.int32) % 7) + 1
    huge = synth.Instance(n=7, row_ptr=row_ptr, lit=lit, ctype=np.zeros(m, np.int8), param=np.zeros(m, np.int32))
    hp = pcls.Problem.from_instance(huge)
    Xh = hp.new_state(1)
    oh = torch.zeros(m, dtype=torch.float32, device=hp.device)
    assert L.pcls_constraint_grad_stats_noalloc(hp.handle, 1, pcls._tptr(Xh), pcls._tptr(oh),
                                                pcls._stream()) == pcls.PCLS_E_UNSUPPORTED
    assert b"static scratch" in L.pcls_last_error()
