"""FP64 reference of the restart-proposal network (plain PyTorch CPU ops).

TEST INFRASTRUCTURE. Only tests may import this module; it shares no code with
the product (features and message passing are written here from their
definition, not imported).

Definition (hidden width 64, three rounds):
    f_v = [deg/8, pos/8, neg/8, 1, 0...] (32 wide); f_c = [type one-hot(7), k/8,
          kappa/k for CARD_GE and EK else 0, parity for XOR else 0, 1, 0...]
    h_v = relu(Ev f_v + ev);  h_c = relu(Ec f_c + ec)
    per round l: h_c' = relu(W1 h_c + bc + (1/k_c) sum_{i in c} W_{s_i} h_{v_i})
                 h_v' = relu(W2 h_v + bv + (1/deg_v) sum_{(c,i): v_i = v} U_{s_i} h_c')
    with W_{+} = Wpn[:64], W_{-} = Wpn[64:], U likewise from Upn;
    x_hat = tanh(wo . h_v + bo).
Every product is FP64 with the parameters exactly as given: a network whose
weight matrices are held in bf16 is evaluated by passing the bf16 values.
"""
from __future__ import annotations

import numpy as np
import torch

HID, FEAT, LAYERS = 64, 32, 3


def spec():
    s = [("Ev", (HID, FEAT)), ("ev", (HID,)), ("Ec", (HID, FEAT)), ("ec", (HID,))]
    for l in range(LAYERS):
        s += [(f"W1_{l}", (HID, HID)), (f"bc_{l}", (HID,)), (f"Wpn_{l}", (2 * HID, HID)),
              (f"W2_{l}", (HID, HID)), (f"bv_{l}", (HID,)), (f"Upn_{l}", (2 * HID, HID))]
    return s + [("wo", (HID,)), ("bo", (1,))]


def unflatten(flat):
    out, o = {}, 0
    for name, shape in spec():
        cnt = int(np.prod(shape))
        out[name] = torch.tensor(np.asarray(flat[o:o + cnt], np.float64).reshape(shape), requires_grad=True)
        o += cnt
    return out


def features(n, row_ptr, lit, ctype, param):
    m = len(row_ptr) - 1
    fv = np.zeros((n, FEAT))
    fc = np.zeros((m, FEAT))
    for c in range(m):
        k = row_ptr[c + 1] - row_ptr[c]
        fc[c, int(ctype[c])] = 1.0
        fc[c, 7] = k / 8.0
        if int(ctype[c]) in (2, 6):
            fc[c, 8] = param[c] / k
        if int(ctype[c]) == 1:
            fc[c, 9] = param[c]
        fc[c, 10] = 1.0
        for i in range(row_ptr[c], row_ptr[c + 1]):
            v = abs(int(lit[i])) - 1
            fv[v, 0] += 1.0 / 8.0
            fv[v, 1 if lit[i] > 0 else 2] += 1.0 / 8.0
    fv[:, 3] = 1.0
    return torch.tensor(fv), torch.tensor(fc)


def forward(instances, params):
    """x_hat for the disjoint union of instances (each: n, row_ptr, lit, ctype, param)."""

    def lin(x, W):
        return x @ W.T

    fvs, fcs, cons, vars_, signs = [], [], [], [], []
    voff = coff = 0
    for (n, row_ptr, lit, ctype, param) in instances:
        fv, fc = features(n, row_ptr, lit, ctype, param)
        fvs.append(fv)
        fcs.append(fc)
        for c in range(len(row_ptr) - 1):
            for i in range(row_ptr[c], row_ptr[c + 1]):
                cons.append(coff + c)
                vars_.append(voff + abs(int(lit[i])) - 1)
                signs.append(1 if lit[i] > 0 else -1)
        voff += n
        coff += len(row_ptr) - 1
    Fv, Fc = torch.cat(fvs), torch.cat(fcs)
    con = torch.tensor(cons, dtype=torch.long)
    var = torch.tensor(vars_, dtype=torch.long)
    pos = torch.tensor(signs) > 0
    Nv, Nc = Fv.shape[0], Fc.shape[0]
    k = torch.zeros(Nc, dtype=torch.float64).index_add_(0, con, torch.ones(len(cons), dtype=torch.float64))
    deg = torch.zeros(Nv, dtype=torch.float64).index_add_(0, var, torch.ones(len(vars_), dtype=torch.float64))
    hv = torch.relu(lin(Fv, params["Ev"]) + params["ev"])
    hc = torch.relu(lin(Fc, params["Ec"]) + params["ec"])
    for l in range(LAYERS):
        # [W_+; W_-] h_v for every variable, then the sign-selected half per literal
        Pm = lin(hv, params[f"Wpn_{l}"])
        msg_src = torch.where(pos[:, None], Pm[var, :HID], Pm[var, HID:])
        msg = torch.zeros(Nc, HID, dtype=torch.float64).index_add(0, con, msg_src) / k.clamp(min=1)[:, None]
        hc = torch.relu(lin(hc, params[f"W1_{l}"]) + params[f"bc_{l}"] + msg)
        Qm = lin(hc, params[f"Upn_{l}"])
        back_src = torch.where(pos[:, None], Qm[con, :HID], Qm[con, HID:])
        back = torch.zeros(Nv, HID, dtype=torch.float64).index_add(0, var, back_src) / deg.clamp(min=1)[:, None]
        hv = torch.relu(lin(hv, params[f"W2_{l}"]) + params[f"bv_{l}"] + back)
    return torch.tanh(hv @ params["wo"] + params["bo"])


def mse_and_grads(instances, flat, labels):
    """Loss mean (x_hat - y)^2 and the gradient of every parameter (flat, spec order)."""
    params = unflatten(flat)
    xhat = forward(instances, params)
    y = torch.tensor(np.concatenate(labels), dtype=torch.float64)
    loss = ((xhat - y) ** 2).mean()
    loss.backward()
    g = np.concatenate([params[name].grad.detach().numpy().reshape(-1) for name, _ in spec()])
    return float(loss.detach()), xhat.detach().numpy(), g
