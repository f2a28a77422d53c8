"""Learned restart initialiser: a message-passing network on the
variable-constraint graph that proposes starting points for the restarts.

The network (hidden width 64, three rounds of messages):
    h_v^0 = relu(E_v f_v + e_v)          h_c^0 = relu(E_c f_c + e_c)
    per round:  h_c <- relu(W1 h_c + b_c + mean_{i in c} Wp/Wn h_{v_i})   (Wp for a positive
                                                                          literal, Wn negated)
                h_v <- relu(W2 h_v + b_v + mean_{c owns v} Up/Un h_c)
    x_hat_v = tanh(w . h_v + b)
Variable features: degree, positive and negative occurrence counts; constraint
features: type one-hot, length, kappa / k (cardinality, exactly-k) or parity.

It is trained on assignments the plain search finds (labels: the mean corner of
the restarts with the fewest violations, a soft marginal in [-1, 1]) with a
mean-squared error, and proposes x0_r = clip(gamma x_hat + sigma u_r, -1, 1),
u_r uniform in [-1, 1).  Uniform initialisation is the fallback whenever the
network is missing or produces a non-finite value.

Every forward, backward and optimiser step runs in the library's kernels
(include/pcls_mpnn.h); this module allocates memory (torch) and sequences calls.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from . import pcls

HID = 64
FEAT = 32
LAYERS = 3
N_TYPES = 7

_bound = False


def _lib():
    global _bound
    L = pcls.load_library()
    if not _bound:
        i32, vp, sz, f32 = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float
        L.pcls_mpnn_gemm.restype = i32
        L.pcls_mpnn_gemm.argtypes = [vp, i32, i32, i32, vp, i32, i32, vp, vp, i32, i32, vp, vp]
        L.pcls_mpnn_gemm_tn_scratch.restype = sz
        L.pcls_mpnn_gemm_tn_scratch.argtypes = [i32, i32, i32]
        L.pcls_mpnn_gemm_tn.restype = i32
        L.pcls_mpnn_gemm_tn.argtypes = [vp, i32, vp, i32, i32, i32, i32, vp, i32, vp, sz, vp]
        L.pcls_mpnn_gather.restype = i32
        L.pcls_mpnn_gather.argtypes = [vp, vp, vp, i32, vp, i32, vp, i32, vp, i32, vp]
        L.pcls_mpnn_relu_grad.restype = i32
        L.pcls_mpnn_relu_grad.argtypes = [vp, vp, vp, i32, vp]
        L.pcls_mpnn_colsum_scratch.restype = sz
        L.pcls_mpnn_colsum_scratch.argtypes = [i32]
        L.pcls_mpnn_colsum.restype = i32
        L.pcls_mpnn_colsum.argtypes = [vp, i32, i32, vp, i32, vp, sz, vp]
        L.pcls_mpnn_head_forward.restype = i32
        L.pcls_mpnn_head_forward.argtypes = [vp, i32, vp, vp, vp, vp]
        L.pcls_mpnn_head_backward.restype = i32
        L.pcls_mpnn_head_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.pcls_mpnn_head_grad_scratch.restype = sz
        L.pcls_mpnn_head_grad_scratch.argtypes = [i32]
        L.pcls_mpnn_head_grad.restype = i32
        L.pcls_mpnn_head_grad.argtypes = [vp, vp, i32, vp, i32, vp, sz, vp]
        L.pcls_mpnn_propose.restype = i32
        L.pcls_mpnn_propose.argtypes = [vp, i32, vp, i32, f32, f32, vp, vp]
        L.pcls_mpnn_mse_scratch.restype = sz
        L.pcls_mpnn_mse_scratch.argtypes = [i32]
        L.pcls_mpnn_mse.restype = i32
        L.pcls_mpnn_mse.argtypes = [vp, vp, i32, vp, vp, vp]
        L.pcls_mpnn_adam.restype = i32
        L.pcls_mpnn_adam.argtypes = [vp, vp, vp, vp, i32, f32, f32, f32, f32, i32, f32, vp, vp]
        L.pcls_mpnn_to_bf16.restype = i32
        L.pcls_mpnn_to_bf16.argtypes = [vp, vp, i32, vp]
        L.pcls_mpnn_last_error.restype = ctypes.c_char_p
        _bound = True
    return L


MPNN_EXPORTS = ["pcls_mpnn_gemm", "pcls_mpnn_gemm_tn_scratch", "pcls_mpnn_gemm_tn", "pcls_mpnn_gather",
                "pcls_mpnn_relu_grad", "pcls_mpnn_colsum_scratch", "pcls_mpnn_colsum", "pcls_mpnn_head_forward",
                "pcls_mpnn_head_backward", "pcls_mpnn_head_grad_scratch", "pcls_mpnn_head_grad",
                "pcls_mpnn_propose", "pcls_mpnn_mse_scratch", "pcls_mpnn_mse", "pcls_mpnn_adam",
                "pcls_mpnn_to_bf16", "pcls_mpnn_last_error"]


def _ck(status):
    if status != 0:
        msg = _lib().pcls_mpnn_last_error()
        raise pcls.PclsError(status, msg.decode() if msg else "")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    return pcls._stream()


# ------------------------------------------------------------------ kernels

def gemm(A, lda, N, K, W, M, trans_w, bias, Y, ldy, beta=0, Y_relu=None):
    _ck(_lib().pcls_mpnn_gemm(_p(A), lda, N, K, _p(W), M, trans_w, _p(bias), _p(Y), ldy, beta, _p(Y_relu), _s()))


class Scratch:
    def __init__(self, device):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        import torch
        if self.buf is None or self.buf.numel() * 4 < nbytes:
            self.buf = torch.empty((nbytes + 3) // 4 + 64, dtype=torch.float32, device=self.device)
        return self.buf, self.buf.numel() * 4


def gemm_tn(dZ, ldz, X, ldx, N, M, K, dW, scratch: Scratch, accumulate=0):
    buf, nb = scratch.get(_lib().pcls_mpnn_gemm_tn_scratch(N, M, K))
    _ck(_lib().pcls_mpnn_gemm_tn(_p(dZ), ldz, _p(X), ldx, N, M, K, _p(dW), accumulate, _p(buf), nb, _s()))


def gather(ptr, idx, w, rows, In, ld_in, Out, ld_out, H_relu, mode):
    _ck(_lib().pcls_mpnn_gather(_p(ptr), _p(idx), _p(w), rows, _p(In), ld_in, _p(Out), ld_out, _p(H_relu), mode,
                                _s()))


def relu_grad(dH, Z, dZ):
    _ck(_lib().pcls_mpnn_relu_grad(_p(dH), _p(Z), _p(dZ), dZ.numel(), _s()))


def colsum(X, ld, N, out, scratch: Scratch, accumulate=0):
    buf, nb = scratch.get(_lib().pcls_mpnn_colsum_scratch(N))
    _ck(_lib().pcls_mpnn_colsum(_p(X), ld, N, _p(out), accumulate, _p(buf), nb, _s()))


def head_forward(H, N, w, b, xhat):
    _ck(_lib().pcls_mpnn_head_forward(_p(H), N, _p(w), _p(b), _p(xhat), _s()))


def head_backward(xhat, dxhat, N, w, dH, dlogit):
    _ck(_lib().pcls_mpnn_head_backward(_p(xhat), _p(dxhat), N, _p(w), _p(dH), _p(dlogit), _s()))


def head_grad(H, dlogit, N, dwb65, scratch: Scratch, accumulate=0):
    buf, nb = scratch.get(_lib().pcls_mpnn_head_grad_scratch(N))
    _ck(_lib().pcls_mpnn_head_grad(_p(H), _p(dlogit), N, _p(dwb65), accumulate, _p(buf), nb, _s()))


def mse(xhat, y, N, dxhat, partial):
    _ck(_lib().pcls_mpnn_mse(_p(xhat), _p(y), N, _p(dxhat), _p(partial), _s()))


def propose(xhat, n, U, R, gamma, sigma, X):
    _ck(_lib().pcls_mpnn_propose(_p(xhat), n, _p(U), R, float(gamma), float(sigma), _p(X), _s()))


# ------------------------------------------------------------------- graphs

def instance_features(inst):
    """Per-variable and per-constraint input features (numpy float32, FEAT wide)."""
    n, m = inst.n, inst.m
    lens = np.diff(inst.row_ptr).astype(np.int64)
    var = np.abs(inst.lit).astype(np.int64) - 1
    neg = inst.lit < 0
    deg = np.bincount(var, minlength=n).astype(np.float32)
    nneg = np.bincount(var[neg], minlength=n).astype(np.float32)
    fv = np.zeros((n, FEAT), np.float32)
    fv[:, 0] = deg / 8.0
    fv[:, 1] = (deg - nneg) / 8.0
    fv[:, 2] = nneg / 8.0
    fv[:, 3] = 1.0
    fc = np.zeros((m, FEAT), np.float32)
    fc[np.arange(m), inst.ctype.astype(np.int64)] = 1.0
    fc[:, N_TYPES] = lens / 8.0
    prm = inst.param.astype(np.float32)
    frac = np.where(np.isin(inst.ctype, (2, 6)), prm / np.maximum(lens, 1), 0.0)
    fc[:, N_TYPES + 1] = frac
    fc[:, N_TYPES + 2] = np.where(inst.ctype == 1, prm, 0.0)
    fc[:, N_TYPES + 3] = 1.0
    return fv, fc


class GraphBatch:
    """Disjoint union of instances as device CSR structures in both directions.

    Constraint-major: cptr / cidx = (variable << 1) | negated, with forward
    weights 1/k_c and transposed weights 1/deg_v.  Variable-major: vptr / vidx =
    (constraint << 1) | negated, forward weights 1/deg_v, transposed 1/k_c."""

    def __init__(self, instances, device):
        import torch
        self.instances = list(instances)
        self.var_off = np.cumsum([0] + [i.n for i in self.instances])
        self.con_off = np.cumsum([0] + [i.m for i in self.instances])
        Nv, Nc = int(self.var_off[-1]), int(self.con_off[-1])
        fvs, fcs, cptr, cidx, cv, cneg = [], [], [0], [], [], []
        for k, inst in enumerate(self.instances):
            fv, fc = instance_features(inst)
            fvs.append(fv)
            fcs.append(fc)
            cptr.extend((inst.row_ptr[1:] + cptr[-1]).tolist())
            v = np.abs(inst.lit).astype(np.int64) - 1 + self.var_off[k]
            cv.append(v)
            cneg.append((inst.lit < 0).astype(np.int64))
        cptr = np.array(cptr, np.int64)
        cv = np.concatenate(cv) if cv else np.zeros(0, np.int64)
        cneg = np.concatenate(cneg) if cneg else np.zeros(0, np.int64)
        L = len(cv)
        con_of = np.repeat(np.arange(Nc), np.diff(cptr))
        klen = np.diff(cptr).astype(np.float64)
        deg = np.bincount(cv, minlength=Nv).astype(np.float64)
        order = np.argsort(cv, kind="stable")
        vptr = np.zeros(Nv + 1, np.int64)
        np.cumsum(np.bincount(cv, minlength=Nv), out=vptr[1:])
        self.Nv, self.Nc, self.L = Nv, Nc, L
        t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=device)  # noqa: E731
        self.Fv = t(np.concatenate(fvs) if fvs else np.zeros((0, FEAT)), torch.float32)
        self.Fc = t(np.concatenate(fcs) if fcs else np.zeros((0, FEAT)), torch.float32)
        self.cptr = t(cptr, torch.int32)
        self.cidx = t((cv << 1) | cneg, torch.int32)
        self.cw = t(1.0 / klen[con_of], torch.float32)
        self.cw_t = t(1.0 / deg[cv], torch.float32)
        self.vptr = t(vptr, torch.int32)
        self.vidx = t((con_of[order] << 1) | cneg[order], torch.int32)
        self.vw = t(1.0 / deg[cv[order]], torch.float32)
        self.vw_t = t(1.0 / klen[con_of[order]], torch.float32)
        self.device = device

    def slice_vars(self, x, k):
        return x[int(self.var_off[k]):int(self.var_off[k + 1])]


# ------------------------------------------------------------------- params

def param_spec():
    spec = [("Ev", (HID, FEAT)), ("ev", (HID,)), ("Ec", (HID, FEAT)), ("ec", (HID,))]
    for l in range(LAYERS):
        spec += [(f"W1_{l}", (HID, HID)), (f"bc_{l}", (HID,)), (f"Wpn_{l}", (2 * HID, HID)),
                 (f"W2_{l}", (HID, HID)), (f"bv_{l}", (HID,)), (f"Upn_{l}", (2 * HID, HID))]
    spec += [("wo", (HID,)), ("bo", (1,))]
    return spec


class Params:
    """Flat float32 master weights, their bf16 copy, gradients and Adam moments."""

    def __init__(self, device, seed=0, flat=None):
        import torch
        self.spec = param_spec()
        self.offsets = {}
        off = 0
        for name, shape in self.spec:
            cnt = int(np.prod(shape))
            self.offsets[name] = (off, shape)
            off += cnt
        self.count = off
        if flat is None:
            rng = np.random.default_rng(seed)
            flat = np.zeros(off, np.float32)
            for name, shape in self.spec:
                o, _ = self.offsets[name]
                if len(shape) == 2:
                    bound = np.sqrt(6.0 / (shape[0] + shape[1]))
                    flat[o:o + shape[0] * shape[1]] = rng.uniform(-bound, bound, shape[0] * shape[1])
                elif name.startswith(("b", "e")) and name != "bo":
                    flat[o:o + shape[0]] = 0.01
                elif name == "wo":
                    flat[o:o + shape[0]] = rng.uniform(-0.1, 0.1, shape[0])
        self.master = torch.tensor(np.asarray(flat, np.float32), device=device)
        self.bf16 = torch.empty(off, dtype=torch.int16, device=device)
        self.grad = torch.zeros(off, dtype=torch.float32, device=device)
        self.m = torch.zeros(off, dtype=torch.float32, device=device)
        self.v = torch.zeros(off, dtype=torch.float32, device=device)
        self.step_count = 0
        self.sync_bf16()

    def sync_bf16(self):
        _ck(_lib().pcls_mpnn_to_bf16(_p(self.master), _p(self.bf16), self.count, _s()))

    def w(self, name):
        o, shape = self.offsets[name]
        return self.master[o:o + int(np.prod(shape))]

    def wb(self, name):
        o, shape = self.offsets[name]
        return self.bf16[o:o + int(np.prod(shape))]

    def g(self, name):
        o, shape = self.offsets[name]
        return self.grad[o:o + int(np.prod(shape))]

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, weight_decay=0.0):
        self.step_count += 1
        _ck(_lib().pcls_mpnn_adam(_p(self.master), _p(self.grad), _p(self.m), _p(self.v), self.count, lr, b1, b2,
                                  eps, self.step_count, weight_decay, _p(self.bf16), _s()))

    def numpy(self):
        return self.master.detach().cpu().numpy().copy()

    def save(self, path, meta=None):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez(path, flat=self.numpy(), meta=json.dumps(meta or {}))

    @classmethod
    def load(cls, path, device):
        with np.load(path, allow_pickle=False) as z:
            flat = z["flat"]
            meta = json.loads(str(z["meta"]))
        p = cls(device, flat=flat)
        return p, meta


# ------------------------------------------------------------------ network

class MPNN:
    def __init__(self, params: Params):
        self.P = params
        self.scratch = Scratch(params.master.device)

    def forward(self, G: GraphBatch, keep=False):
        import torch
        P, Nv, Nc, dev = self.P, G.Nv, G.Nc, G.device
        e = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)  # noqa: E731
        Zv0, Hv, Zc0, Hc = e(Nv, HID), e(Nv, HID), e(Nc, HID), e(Nc, HID)
        gemm(G.Fv, FEAT, Nv, FEAT, P.wb("Ev"), HID, 0, P.w("ev"), Zv0, HID, 0, Hv)
        gemm(G.Fc, FEAT, Nc, FEAT, P.wb("Ec"), HID, 0, P.w("ec"), Zc0, HID, 0, Hc)
        caches = []
        for l in range(LAYERS):
            Pm, Zc, Hc2, Qm, Zv, Hv2 = e(Nv, 2 * HID), e(Nc, HID), e(Nc, HID), e(Nc, 2 * HID), e(Nv, HID), e(Nv, HID)
            gemm(Hv, HID, Nv, HID, P.wb(f"Wpn_{l}"), 2 * HID, 0, None, Pm, 2 * HID)
            gemm(Hc, HID, Nc, HID, P.wb(f"W1_{l}"), HID, 0, P.w(f"bc_{l}"), Zc, HID)
            gather(G.cptr, G.cidx, G.cw, Nc, Pm, 2 * HID, Zc, HID, Hc2, 0)
            gemm(Hc2, HID, Nc, HID, P.wb(f"Upn_{l}"), 2 * HID, 0, None, Qm, 2 * HID)
            gemm(Hv, HID, Nv, HID, P.wb(f"W2_{l}"), HID, 0, P.w(f"bv_{l}"), Zv, HID)
            gather(G.vptr, G.vidx, G.vw, Nv, Qm, 2 * HID, Zv, HID, Hv2, 0)
            if keep:
                caches.append((Hv, Hc, Zc, Hc2, Zv))
            Hv, Hc = Hv2, Hc2
        xhat = e(Nv)
        head_forward(Hv, Nv, P.w("wo"), P.w("bo"), xhat)
        if keep:
            self._cache = (Zv0, Zc0, caches, Hv, xhat, G)
        return xhat

    def backward(self, dxhat):
        """Gradients of every parameter (written, not accumulated) from dL/dxhat."""
        import torch
        P, sc = self.P, self.scratch
        Zv0, Zc0, caches, HvL, xhat, G = self._cache
        Nv, Nc, dev = G.Nv, G.Nc, G.device
        e = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)  # noqa: E731
        dHv, dlogit = e(Nv, HID), e(Nv)
        head_backward(xhat, dxhat, Nv, P.w("wo"), dHv, dlogit)
        o_wo = P.offsets["wo"][0]
        head_grad(HvL, dlogit, Nv, P.grad[o_wo:o_wo + HID + 1], sc)  # wo and bo are adjacent
        dHc = None
        for l in reversed(range(LAYERS)):
            Hv, Hc, Zc, Hc2, Zv = caches[l]
            dZv = e(Nv, HID)
            relu_grad(dHv, Zv, dZv)
            colsum(dZv, HID, Nv, P.g(f"bv_{l}"), sc)
            gemm_tn(dZv, HID, Hv, HID, Nv, HID, HID, P.g(f"W2_{l}"), sc)
            dHv_in = e(Nv, HID)
            gemm(dZv, HID, Nv, HID, P.wb(f"W2_{l}"), HID, 1, None, dHv_in, HID)
            dQ = e(Nc, 2 * HID)
            gather(G.cptr, G.cidx, G.cw_t, Nc, dZv, HID, dQ, 2 * HID, None, 1)
            gemm_tn(dQ, 2 * HID, Hc2, HID, Nc, 2 * HID, HID, P.g(f"Upn_{l}"), sc)
            if dHc is None:
                dHc = e(Nc, HID)
                gemm(dQ, 2 * HID, Nc, 2 * HID, P.wb(f"Upn_{l}"), HID, 1, None, dHc, HID, 0)
            else:
                gemm(dQ, 2 * HID, Nc, 2 * HID, P.wb(f"Upn_{l}"), HID, 1, None, dHc, HID, 1)
            dZc = e(Nc, HID)
            relu_grad(dHc, Zc, dZc)
            colsum(dZc, HID, Nc, P.g(f"bc_{l}"), sc)
            gemm_tn(dZc, HID, Hc, HID, Nc, HID, HID, P.g(f"W1_{l}"), sc)
            dHc_in = e(Nc, HID)
            gemm(dZc, HID, Nc, HID, P.wb(f"W1_{l}"), HID, 1, None, dHc_in, HID)
            dP = e(Nv, 2 * HID)
            gather(G.vptr, G.vidx, G.vw_t, Nv, dZc, HID, dP, 2 * HID, None, 1)
            gemm_tn(dP, 2 * HID, Hv, HID, Nv, 2 * HID, HID, P.g(f"Wpn_{l}"), sc)
            gemm(dP, 2 * HID, Nv, 2 * HID, P.wb(f"Wpn_{l}"), HID, 1, None, dHv_in, HID, 1)
            dHv, dHc = dHv_in, dHc_in
        dZv0, dZc0 = e(Nv, HID), e(Nc, HID)
        relu_grad(dHv, Zv0, dZv0)
        relu_grad(dHc, Zc0, dZc0)
        colsum(dZv0, HID, Nv, P.g("ev"), sc)
        colsum(dZc0, HID, Nc, P.g("ec"), sc)
        gemm_tn(dZv0, HID, G.Fv, FEAT, Nv, HID, FEAT, P.g("Ev"), sc)
        gemm_tn(dZc0, HID, G.Fc, FEAT, Nc, HID, FEAT, P.g("Ec"), sc)

    def mse_loss_grad(self, xhat, y):
        """dL/dxhat for L = mean (xhat - y)^2; returns (dxhat, loss tensor)."""
        import torch
        N = xhat.numel()
        dx = torch.empty_like(xhat)
        part = torch.empty((N + 255) // 256 + 1, dtype=torch.float32, device=xhat.device)
        mse(xhat, y, N, dx, part)
        return dx, part[: (N + 255) // 256]


# --------------------------------------------------------- labels, training

def cls_labels(instances, restarts=64, steps=500, lr=0.1, seed=0):
    """Soft marginals from the plain search: for each instance, the mean corner
    of the restarts with the fewest violated constraints after `steps` steps."""
    import torch

    from .batch import Batch
    probs = [pcls.Problem.from_instance(i) for i in instances]
    states = []
    for k, p in enumerate(probs):
        X = p.new_state(restarts)
        p.init_restarts(X, restarts, seed + k)
        states.append(X)
    b = Batch(probs, [restarts] * len(probs), states)
    b.step(lr, steps)
    labels, best_unsat = [], []
    for p, X in zip(probs, states):
        assign, unsat, _ = p.extract(X, restarts)
        u = unsat.cpu().numpy()
        sel = u == u.min()
        lab = assign.cpu().numpy()[sel].astype(np.float32).mean(axis=0)
        labels.append(lab)
        best_unsat.append(int(u.min()))
    torch.cuda.synchronize()
    return labels, best_unsat


def train(instances, labels, steps=1500, batch_size=16, lr=2e-3, seed=0, device="cuda", log_every=100,
          params: Params | None = None, log=None):
    import torch
    P = params or Params(device, seed=seed)
    net = MPNN(P)
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(instances))
    batches = []
    for s in range(0, len(order) - batch_size + 1, batch_size):
        idx = order[s:s + batch_size]
        G = GraphBatch([instances[i] for i in idx], device)
        y = torch.tensor(np.concatenate([labels[i] for i in idx]), dtype=torch.float32, device=device)
        batches.append((G, y))
    history = []
    for it in range(steps):
        G, y = batches[it % len(batches)]
        xhat = net.forward(G, keep=True)
        dx, part = net.mse_loss_grad(xhat, y)
        net.backward(dx)
        P.adam(lr=lr)
        if (it + 1) % log_every == 0 or it == 0:
            loss = float(part.sum().item())
            history.append((it + 1, loss))
            if log:
                log(f"train step {it + 1}: loss {loss:.5f}")
    torch.cuda.synchronize()
    return P, history


def predict(P: Params, instances, device="cuda"):
    """x_hat per instance (list of device tensors); None where non-finite."""
    import torch
    G = GraphBatch(instances, device)
    xhat = MPNN(P).forward(G)
    out = []
    for k in range(len(instances)):
        xs = G.slice_vars(xhat, k)
        out.append(xs if bool(torch.isfinite(xs).all()) else None)
    return out


def initial_states(problem, xhat, R, seed, gamma, sigma):
    """Learned proposal x0 = clip(gamma x_hat + sigma u, -1, 1); uniform when x_hat is None."""
    X = problem.new_state(R)
    problem.init_restarts(X, R, seed)
    if xhat is None:
        return X, False
    Xl = problem.new_state(R)
    propose(xhat, problem.n, X, R, gamma, sigma, Xl)
    return Xl, True


def sat_fraction_curves(instances, budgets, R=64, seed=0, P: Params | None = None, gamma=1.0, sigma=0.5,
                        lr=0.1, device="cuda"):
    """Satisfied-constraint fraction (best over restarts and mean over restarts)
    at each cumulative step budget, per instance.  P None = uniform init."""
    probs = [pcls.Problem.from_instance(i, device=device) for i in instances]
    xh = predict(P, instances, device) if P is not None else [None] * len(instances)
    states, used = [], []
    for k, p in enumerate(probs):
        X, u = initial_states(p, xh[k], R, seed + k, gamma, sigma)
        states.append(X)
        used.append(u)
    best = np.zeros((len(instances), len(budgets)))
    mean = np.zeros_like(best)
    done = 0
    for bi, S in enumerate(budgets):
        if S > done:
            from .batch import Batch
            b = Batch(probs, [R] * len(probs), states)
            b.step(lr, S - done)
            done = S
        for k, (p, X) in enumerate(zip(probs, states)):
            _, unsat, _ = p.extract(X, R, want_assign=False)
            u = unsat.cpu().numpy().astype(np.float64)
            best[k, bi] = 1.0 - u.min() / instances[k].m
            mean[k, bi] = 1.0 - u.mean() / instances[k].m
    return {"best": best, "mean": mean, "learned_used": used}


def paired_bootstrap_ci(diff, reps=10000, seed=0, alpha=0.05):
    rng = np.random.default_rng(seed)
    diff = np.asarray(diff, np.float64)
    boots = rng.choice(diff, size=(reps, len(diff)), replace=True).mean(axis=1)
    return float(diff.mean()), float(np.quantile(boots, alpha / 2)), float(np.quantile(boots, 1 - alpha / 2))
