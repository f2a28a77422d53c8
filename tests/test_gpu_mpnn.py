"""Kernels of the learned initialiser: every primitive against float64 torch with
the same bf16-rounded operands, the whole network against the FP64 reference,
training, and the gain of learned over uniform restarts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import mpnn_ref as M  # noqa: E402
from paper_2606_06656_amd import learned as LRN  # noqa: E402
from paper_2606_06656_amd import synth  # noqa: E402
from gpu_util import log  # noqa: E402

DEV = "cuda"


def bf(x):
    return x.to(torch.bfloat16).to(torch.float64)


def to_bits(w32):
    return w32.to(torch.bfloat16).view(torch.int16)


@pytest.mark.parametrize("N,K,M,trans", [(1, 32, 16, 0), (70, 64, 64, 0), (130, 64, 128, 0), (200, 128, 64, 1),
                                         (65, 64, 64, 1), (3, 96, 32, 0)])
def test_gemm(N, K, M, trans):
    log(f"case gemm N={N} K={K} M={M} trans={trans}")
    g = torch.Generator().manual_seed(N * 7 + K)
    A = torch.randn(N, K + 3, generator=g)  # row stride K + 3
    Wshape = (M, K) if trans == 0 else (K, M)
    W = torch.randn(*Wshape, generator=g) * 0.2
    bias = torch.randn(M, generator=g)
    Y0 = torch.randn(N, M + 5, generator=g)
    Ad, Wd = A.to(DEV), to_bits(W.to(DEV))
    Y = Y0.clone().to(DEV)
    Yr = torch.zeros_like(Y)
    LRN.gemm(Ad, K + 3, N, K, Wd, M, trans, bias.to(DEV), Y, M + 5, 1, Yr)
    opW = bf(W).T if trans == 0 else bf(W)
    # A enters as two bf16 parts, hi = bf16(A) and lo = bf16(A - hi); W is bf16
    a = A[:, :K].double()
    ah = bf(a)
    al = bf(a - ah)
    ref = Y0.double().clone()
    ref[:, :M] += ah @ opW + al @ opW + bias.double()
    np.testing.assert_allclose(Y.cpu().double().numpy(), ref.numpy(), rtol=1e-5, atol=1e-4)
    # within about 2^-16 relative per term of the float32 operand times the bf16 weight
    exact = Y0.double().clone()
    exact[:, :M] += a @ opW + bias.double()
    np.testing.assert_allclose(Y.cpu().double().numpy(), exact.numpy(), rtol=1e-4, atol=1e-3)
    np.testing.assert_allclose(Yr[:, :M].cpu().double().numpy(), np.maximum(ref[:, :M].numpy(), 0), rtol=1e-5,
                               atol=1e-4)


@pytest.mark.parametrize("N,M,K", [(1, 16, 16), (100, 64, 64), (2500, 128, 64), (33, 64, 32)])
def test_gemm_tn(N, M, K):
    log(f"case gemm_tn N={N} M={M} K={K}")
    g = torch.Generator().manual_seed(N + M)
    dZ = torch.randn(N, M + 2, generator=g)
    X = torch.randn(N, K + 1, generator=g)
    dW = torch.randn(M, K, generator=g).to(DEV)
    base = dW.clone()
    sc = LRN.Scratch(DEV)
    LRN.gemm_tn(dZ.to(DEV), M + 2, X.to(DEV), K + 1, N, M, K, dW, sc, accumulate=1)
    a, b = dZ[:, :M].double(), X[:, :K].double()
    ah, bh = bf(a), bf(b)
    al, bl = bf(a - ah), bf(b - bh)
    ref = ah.T @ bh + ah.T @ bl + al.T @ bh
    exact = a.T @ b
    np.testing.assert_allclose((dW - base).cpu().double().numpy(), ref.numpy(), rtol=1e-4, atol=1e-3)
    LRN.gemm_tn(dZ.to(DEV), M + 2, X.to(DEV), K + 1, N, M, K, dW, sc, accumulate=0)
    np.testing.assert_allclose(dW.cpu().double().numpy(), ref.numpy(), rtol=1e-4, atol=1e-3)
    # split operands: close to the exact product (about 2^-16 relative per term)
    np.testing.assert_allclose(dW.cpu().double().numpy(), exact.numpy(), rtol=1e-3, atol=2e-3 * np.sqrt(N))


def graph_of(instances):
    return LRN.GraphBatch(instances, DEV)


def test_gather_both_modes():
    insts = [synth.mixed_small(n=40, seed=1, kmax=6, count=50), synth.random_ksat(30, 60, 3, seed=2)]
    G = graph_of(insts)
    log("case gather")
    g = torch.Generator().manual_seed(3)
    Pm = torch.randn(G.Nv, 128, generator=g)
    Z0 = torch.randn(G.Nc, 64, generator=g)
    Z = Z0.clone().to(DEV)
    Hr = torch.zeros_like(Z)
    LRN.gather(G.cptr, G.cidx, G.cw, G.Nc, Pm.to(DEV), 128, Z, 64, Hr, 0)
    # reference from the raw instance arrays
    ref = Z0.double().clone()
    coff = voff = 0
    for inst in insts:
        for c in range(inst.m):
            lits = inst.lit[inst.row_ptr[c]:inst.row_ptr[c + 1]]
            for l in lits:
                v = voff + abs(int(l)) - 1
                ref[coff + c] += Pm[v, (0 if l > 0 else 64):(64 if l > 0 else 128)].double() / len(lits)
        coff += inst.m
        voff += inst.n
    np.testing.assert_allclose(Z.cpu().double().numpy(), ref.numpy(), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(Hr.cpu().double().numpy(), np.maximum(ref.numpy(), 0), rtol=1e-5, atol=1e-5)
    # transposed: Out[v][half] = sum over occurrences dZ[c] / k_c
    dZ = torch.randn(G.Nc, 64, generator=g)
    out = torch.zeros(G.Nv, 128, device=DEV)
    LRN.gather(G.vptr, G.vidx, G.vw_t, G.Nv, dZ.to(DEV), 64, out, 128, None, 1)
    ref2 = torch.zeros(G.Nv, 128, dtype=torch.float64)
    coff = voff = 0
    for inst in insts:
        for c in range(inst.m):
            lits = inst.lit[inst.row_ptr[c]:inst.row_ptr[c + 1]]
            for l in lits:
                v = voff + abs(int(l)) - 1
                h = 0 if l > 0 else 64
                ref2[v, h:h + 64] += dZ[coff + c].double() / len(lits)
        coff += inst.m
        voff += inst.n
    np.testing.assert_allclose(out.cpu().double().numpy(), ref2.numpy(), rtol=1e-5, atol=1e-5)


def test_head_mse_colsum_adam():
    log("case head/mse/colsum/adam")
    g = torch.Generator().manual_seed(11)
    N = 1500
    H = torch.randn(N, 64, generator=g)
    w = torch.randn(64, generator=g) * 0.1
    b = torch.tensor([0.3])
    Hd, wd, bd = H.to(DEV), w.to(DEV), b.to(DEV)
    xhat = torch.empty(N, device=DEV)
    LRN.head_forward(Hd, N, wd, bd, xhat)
    ref = torch.tanh(H.double() @ w.double() + 0.3)
    np.testing.assert_allclose(xhat.cpu().double().numpy(), ref.numpy(), atol=2e-6)
    y = torch.rand(N, generator=g) * 2 - 1
    dx = torch.empty(N, device=DEV)
    part = torch.empty(N // 256 + 2, device=DEV)
    LRN.mse(xhat, y.to(DEV), N, dx, part)
    loss_ref = ((ref - y.double()) ** 2).mean()
    assert part[: (N + 255) // 256].sum().item() == pytest.approx(float(loss_ref), rel=1e-5)
    np.testing.assert_allclose(dx.cpu().double().numpy(), (2 * (ref - y.double()) / N).numpy(), atol=1e-8)
    dH = torch.empty(N, 64, device=DEV)
    dlogit = torch.empty(N, device=DEV)
    LRN.head_backward(xhat, dx, N, wd, dH, dlogit)
    dl_ref = dx.cpu().double() * (1 - xhat.cpu().double() ** 2)
    np.testing.assert_allclose(dlogit.cpu().double().numpy(), dl_ref.numpy(), rtol=1e-5, atol=1e-10)
    np.testing.assert_allclose(dH.cpu().double().numpy(), (dl_ref[:, None] * w.double()).numpy(), rtol=1e-5,
                               atol=1e-10)
    sc = LRN.Scratch(DEV)
    dwb = torch.zeros(65, device=DEV)
    LRN.head_grad(Hd, dlogit, N, dwb, sc)
    np.testing.assert_allclose(dwb[:64].cpu().double().numpy(), (H.double().T @ dl_ref).numpy(), rtol=1e-4,
                               atol=1e-7)
    assert dwb[64].item() == pytest.approx(float(dl_ref.sum()), rel=1e-4, abs=1e-7)
    cs = torch.zeros(64, device=DEV)
    LRN.colsum(Hd, 64, N, cs, sc)
    np.testing.assert_allclose(cs.cpu().double().numpy(), H.double().sum(0).numpy(), rtol=1e-5, atol=1e-4)
    # Adam: two steps against the textbook update
    P = LRN.Params(DEV, seed=1)
    p0 = P.master.cpu().double().clone()
    grads = [torch.randn(P.count, generator=g) for _ in range(2)]
    m = torch.zeros(P.count, dtype=torch.float64)
    v = torch.zeros(P.count, dtype=torch.float64)
    p = p0.clone()
    for t, gr in enumerate(grads, start=1):
        P.grad.copy_(gr.to(DEV))
        P.adam(lr=1e-2)
        m = 0.9 * m + 0.1 * gr.double()
        v = 0.999 * v + 0.001 * gr.double() ** 2
        p = p - 1e-2 * (m / (1 - 0.9 ** t)) / (torch.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    np.testing.assert_allclose(P.master.cpu().double().numpy(), p.numpy(), atol=2e-6)
    assert torch.equal(P.bf16.cpu(), P.master.cpu().to(torch.bfloat16).view(torch.int16))


def oracle_tuple(inst):
    return (inst.n, inst.row_ptr, inst.lit, inst.ctype, inst.param)


def bf16_matrices(flat):
    """The network the kernels hold: weight matrices rounded to bf16 (round to
    nearest even, as the library's copy), biases and the output head in float32."""
    out = np.array(flat, np.float64)
    o = 0
    for name, shape in M.spec():
        cnt = int(np.prod(shape))
        if len(shape) == 2:
            out[o:o + cnt] = torch.tensor(out[o:o + cnt]).to(torch.bfloat16).double().numpy()
        o += cnt
    return out


def test_network_forward_and_gradients_match_reference():
    """The GPU network (bf16 weight matrices, float32 activations entering the
    MFMA as two bf16 parts, float32 accumulation) against the exact FP64
    network with the same bf16 weights: forward to 1e-4, every parameter
    tensor's gradient to 1e-3 relative (16-bit operands: about 2^-16 per
    product, float32 sums of at most 128 terms).  Against the network with the
    unrounded float32 master weights the gap is the bf16 rounding of the
    weights themselves, which the configuration prescribes: the exact FP64
    network with the bf16 weights shows the same gap, tensor by tensor, to
    within 1e-3."""
    insts = [synth.mixed_small(n=60, seed=5, kmax=7, count=90), synth.random_ksat(50, 200, 3, seed=6)]
    log("case mpnn full")
    P = LRN.Params(DEV, seed=3)
    G = graph_of(insts)
    net = LRN.MPNN(P)
    xhat = net.forward(G, keep=True)
    tuples = [oracle_tuple(i) for i in insts]
    master = P.master.cpu().double().numpy()
    held = bf16_matrices(master)
    with torch.no_grad():
        xr = M.forward(tuples, M.unflatten(held)).numpy()
    np.testing.assert_allclose(xhat.cpu().double().numpy(), xr, atol=1e-4)
    y = [np.random.default_rng(7 + k).uniform(-1, 1, i.n) for k, i in enumerate(insts)]
    yt = torch.tensor(np.concatenate(y), dtype=torch.float32, device=DEV)
    dx, part = net.mse_loss_grad(xhat, yt)
    net.backward(dx)
    g = P.grad.cpu().double().numpy()

    def per_tensor(g_ref, g_got=g):
        rel = {}
        for name, shape in M.spec():
            o, _ = P.offsets[name]
            cnt = int(np.prod(shape))
            a, r = g_got[o:o + cnt], g_ref[o:o + cnt]
            rel[name] = float(np.linalg.norm(a - r) / (np.linalg.norm(r) + 1e-12))
        return rel

    loss_h, _, g_h = M.mse_and_grads(tuples, held, y)
    assert part.sum().item() == pytest.approx(loss_h, rel=1e-4)
    rel_h = per_tensor(g_h)
    log(f"per-tensor relative gradient error vs the FP64 network with the bf16 weights: {rel_h}")
    assert max(rel_h.values()) <= 1e-3, rel_h
    loss_m, _, g_m = M.mse_and_grads(tuples, master, y)
    assert part.sum().item() == pytest.approx(loss_m, rel=1e-2)
    rel_m = per_tensor(g_m)
    rel_w = per_tensor(g_m, g_h)  # the same gap, exact arithmetic: weight rounding alone
    log(f"per-tensor gap to the float32-master network: GPU {rel_m}; FP64 with bf16 weights {rel_w}")
    assert all(abs(rel_m[k] - rel_w[k]) <= 1e-3 for k in rel_m), (rel_m, rel_w)
    cos = g @ g_m / (np.linalg.norm(g) * np.linalg.norm(g_m))
    assert cos > 0.99, cos


def test_training_reduces_loss():
    train = [synth.c5_train(i) for i in range(32)]
    log("case mpnn training")
    labels, _ = LRN.cls_labels(train, restarts=32, steps=200, seed=1)
    P, hist = LRN.train(train, labels, steps=120, batch_size=8, lr=3e-3, log_every=20)
    assert hist[-1][1] < 0.85 * hist[0][1], hist


def test_learned_init_beats_uniform_at_equal_budget():
    """Train briefly on CLS-labelled 3-SAT (n = 200, ratio 4.2), then compare the
    satisfied fraction of learned and uniform restarts on held-out instances."""
    train = [synth.c5_train(i) for i in range(96)]
    log("case learned vs uniform")
    labels, _ = LRN.cls_labels(train, restarts=64, steps=300, seed=2)
    P, _ = LRN.train(train, labels, steps=400, batch_size=16, lr=2e-3)
    evals = [synth.c5_eval(200, i) for i in range(16)]
    budgets = [0, 10]
    lrn = LRN.sat_fraction_curves(evals, budgets, R=64, seed=50, P=P, gamma=1.0, sigma=0.5)
    uni = LRN.sat_fraction_curves(evals, budgets, R=64, seed=50, P=None)
    assert all(lrn["learned_used"])
    for bi, S in enumerate(budgets):
        d = lrn["mean"][:, bi] - uni["mean"][:, bi]
        mean, lo, hi = LRN.paired_bootstrap_ci(d)
        log(f"budget {S}: mean-over-R gain {mean:.4f} CI [{lo:.4f}, {hi:.4f}]")
        assert lo > 0, (S, mean, lo, hi)
