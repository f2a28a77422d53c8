"""Seeded synthetic instance generators.

These build the formulas the benchmark and the tests run on.  They hold none
of the objective's arithmetic: only random structure (which variables, which
signs, which constraint types and lengths), drawn with NumPy's PCG64.  Both the
HIP path and the oracle consume their output.

A formula is returned as an `Instance`: `n` variables, constraints in CSR form
(`row_ptr[m+1]`, `lit[L]` with +v / -v for a positive / negated literal over
1-based variable v), a type code and a parameter per constraint, and weights.
Within every constraint the variables are distinct.

Type codes: 0 OR, 1 XOR (param = parity of the number of true literals; 1 is
the usual odd parity), 2 CARD_GE (param = kappa), 3 NAE, 4 EO, 5 AMO,
6 EK (param = kappa).

The workload shapes follow the case studies of the paper where it gives them
(random 3-SAT at the clause/variable ratio of about 4.26, "Hard Random 3-SAT")
and otherwise the configurations this project measures: a mixed
clause/XOR/cardinality instance, a long-support stress instance with
geometrically distributed lengths, a batch of uneven instances, and the
3-SAT training/evaluation sets of the learned initialiser.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OR, XOR, CARD_GE, NAE, EO, AMO, EK = range(7)


@dataclass
class Instance:
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    lit: np.ndarray      # int32 [L]
    ctype: np.ndarray    # int8 [m]
    param: np.ndarray    # int32 [m]
    weight: np.ndarray | None = None  # float32 [m] or None (all 1.0)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def L(self) -> int:
        return int(self.row_ptr[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _distinct_vars(rng: np.random.Generator, n: int, k: int, count: int) -> np.ndarray:
    """count rows of k distinct variables in [0, n), uniformly (rejection)."""
    if k > n:
        raise ValueError(f"constraint length {k} exceeds n={n}")
    if count == 0:
        return np.zeros((0, k), np.int64)
    if k * 4 > n:  # dense draw: per-row permutation prefix
        return np.stack([rng.permutation(n)[:k] for _ in range(count)])
    out = rng.integers(0, n, size=(count, k))
    while True:
        s = np.sort(out, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if len(bad) == 0:
            return out
        out[bad] = rng.integers(0, n, size=(len(bad), k))


def _signs(rng: np.random.Generator, shape) -> np.ndarray:
    return np.where(rng.random(shape) < 0.5, -1, 1)


def _assemble(n, groups, name="", meta=None) -> Instance:
    """groups: list of (vars[count,k] 0-based, signs[count,k], ctype, params[count])."""
    lits, lengths, types, params = [], [], [], []
    for vars_, signs, ctype, prm in groups:
        count, k = vars_.shape
        lits.append(((vars_ + 1) * signs).astype(np.int32).reshape(-1))
        lengths.append(np.full(count, k, np.int64))
        types.append(np.full(count, ctype, np.int8))
        params.append(np.asarray(prm, np.int32).reshape(-1))
    lengths = np.concatenate(lengths) if lengths else np.zeros(0, np.int64)
    row_ptr = np.zeros(len(lengths) + 1, np.int32)
    np.cumsum(lengths, out=row_ptr[1:])
    lit = np.concatenate(lits) if lits else np.zeros(0, np.int32)
    return Instance(n=n, row_ptr=row_ptr, lit=lit,
                    ctype=np.concatenate(types) if types else np.zeros(0, np.int8),
                    param=np.concatenate(params) if params else np.zeros(0, np.int32),
                    name=name, meta=meta or {})


def random_ksat(n: int, m: int, k: int = 3, seed: int = 0, name: str = "") -> Instance:
    """Uniform random k-SAT: distinct variables per clause, signs +/-1 with p = 1/2."""
    rng = np.random.default_rng(seed)
    v = _distinct_vars(rng, n, k, m)
    s = _signs(rng, v.shape)
    return _assemble(n, [(v, s, OR, np.zeros(m))], name or f"{k}sat_n{n}_m{m}_s{seed}",
                     {"seed": seed})


def c1_3sat(seed: int = 0) -> Instance:
    """Random 3-SAT, n = 50, m = 213 (ratio 4.26)."""
    return random_ksat(50, 213, 3, seed, name=f"c1_3sat_n50_m213_s{seed}")


def c2_mixed(seed: int = 2, n: int = 2000, n_or: int = 6000, n_xor: int = 600, n_card: int = 200) -> Instance:
    """Mixed symmetric PB instance: 3-clauses, XOR-5 with a random parity bit over
    positive literals, and 'at least 3 of 8' cardinality constraints."""
    rng = np.random.default_rng(seed)
    v_or = _distinct_vars(rng, n, 3, n_or)
    s_or = _signs(rng, v_or.shape)
    v_x = _distinct_vars(rng, n, 5, n_xor)
    s_x = np.ones_like(v_x)
    b_x = rng.integers(0, 2, size=n_xor)
    v_c = _distinct_vars(rng, n, 8, n_card)
    s_c = _signs(rng, v_c.shape)
    return _assemble(n, [(v_or, s_or, OR, np.zeros(n_or)), (v_x, s_x, XOR, b_x),
                         (v_c, s_c, CARD_GE, np.full(n_card, 3))],
                     f"c2_mixed_n{n}_s{seed}", {"seed": seed})


def truncated_geometric(rng, count, lo=3, hi=256, q=0.9) -> np.ndarray:
    """k in [lo, hi] with P(k) proportional to q^(k - lo)."""
    ks = np.arange(lo, hi + 1)
    p = q ** (ks - lo)
    p /= p.sum()
    return rng.choice(ks, size=count, p=p)


def _long_group(rng, n, ctype, k, count):
    v = _distinct_vars(rng, n, k, count)
    s = _signs(rng, v.shape)
    if ctype == XOR:
        prm = np.ones(count)
    elif ctype == CARD_GE:
        prm = np.full(count, (k + 1) // 2)
    else:
        prm = np.zeros(count)
    return (v, s, ctype, prm)


def c3_long(seed: int = 3, n: int = 20000, m: int = 40000, lo: int = 3, hi: int = 256) -> Instance:
    """Long-support stress: lengths truncated-geometric on [3, 256] (mean about 12),
    type uniform over OR / XOR (odd) / CARD >= ceil(k/2) / NAE, random signs."""
    rng = np.random.default_rng(seed)
    ks = truncated_geometric(rng, m, lo, hi)
    types = rng.choice([OR, XOR, CARD_GE, NAE], size=m)
    groups = []
    for k in np.unique(ks):
        for t in (OR, XOR, CARD_GE, NAE):
            cnt = int(np.sum((ks == k) & (types == t)))
            if cnt:
                groups.append(_long_group(rng, n, t, int(k), cnt))
    inst = _assemble(n, groups, f"c3_long_n{n}_m{m}_s{seed}", {"seed": seed})
    return _shuffle_constraints(inst, rng)


def c3_forced_long(seed: int = 31, n: int = 20000, per_type: int = 64,
                   lengths=(64, 96, 128, 192, 256)) -> Instance:
    """Forced long constraints: per_type of each type at each length."""
    rng = np.random.default_rng(seed)
    groups = [_long_group(rng, n, t, k, per_type) for k in lengths for t in (OR, XOR, CARD_GE, NAE)]
    return _assemble(n, groups, f"c3_forced_long_n{n}_s{seed}", {"seed": seed})


def _shuffle_constraints(inst: Instance, rng) -> Instance:
    perm = rng.permutation(inst.m)
    rows = [inst.lit[inst.row_ptr[c]:inst.row_ptr[c + 1]] for c in perm]
    lengths = np.array([len(r) for r in rows], np.int64)
    row_ptr = np.zeros(inst.m + 1, np.int32)
    np.cumsum(lengths, out=row_ptr[1:])
    return Instance(inst.n, row_ptr, np.concatenate(rows).astype(np.int32), inst.ctype[perm].copy(),
                    inst.param[perm].copy(), None if inst.weight is None else inst.weight[perm].copy(),
                    inst.name, inst.meta)


def c4_instance(i: int) -> Instance:
    """Instance i of the uneven batch: n log-uniform in [100, 10^4], 3-clauses at
    ratio 4.2 plus XOR-5 at 0.1 n (odd parity, random signs)."""
    seed = 4000 + i
    rng = np.random.default_rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(100), math.log(10000)))))
    m_or, m_x = int(round(4.2 * n)), int(round(0.1 * n))
    v_or = _distinct_vars(rng, n, 3, m_or)
    s_or = _signs(rng, v_or.shape)
    v_x = _distinct_vars(rng, n, 5, m_x)
    s_x = _signs(rng, v_x.shape)
    return _assemble(n, [(v_or, s_or, OR, np.zeros(m_or)), (v_x, s_x, XOR, np.ones(m_x))],
                     f"c4_{i}_n{n}", {"seed": seed})


def c4_batch(count: int = 256) -> list[Instance]:
    return [c4_instance(i) for i in range(count)]


def c5_train(i: int) -> Instance:
    return random_ksat(200, 840, 3, 10000 + i, name=f"c5_train_{i}")


def c5_eval(n: int, i: int) -> Instance:
    return random_ksat(n, int(round(4.2 * n)), 3, 20000 + i, name=f"c5_eval_n{n}_{i}")


def planted(n: int, counts: dict, seed: int = 0, k_range=(3, 8)) -> tuple[Instance, np.ndarray]:
    """Random constraints all satisfied by a hidden corner z (+1 False, -1 True).

    counts maps a type code to a number of constraints.  Lengths are uniform in
    k_range.  Constraints the hidden corner violates are redrawn (OR, NAE,
    CARD_GE with kappa = ceil(k/2)); XOR takes the parity z gives; EO / AMO / EK
    are built around the true literals z implies.
    """
    rng = np.random.default_rng(seed)
    z = np.where(rng.random(n) < 0.5, -1, 1)
    rows, types, params = [], [], []
    for ctype, count in counts.items():
        for _ in range(count):
            k = int(rng.integers(k_range[0], k_range[1] + 1))
            while True:
                v = rng.choice(n, size=k, replace=False)
                s = _signs(rng, k)
                truth = (s * z[v]) == -1
                t = int(truth.sum())
                prm = 0
                if ctype == OR:
                    ok = t >= 1
                elif ctype == NAE:
                    ok = 0 < t < k
                elif ctype == CARD_GE:
                    prm = (k + 1) // 2
                    ok = t >= prm
                elif ctype == XOR:
                    prm, ok = t % 2, True
                elif ctype == EO:
                    ok = t == 1
                elif ctype == AMO:
                    ok = t <= 1
                elif ctype == EK:
                    prm, ok = t, True
                else:
                    raise ValueError(ctype)
                if ok:
                    break
            rows.append(((v + 1) * s).astype(np.int32))
            types.append(ctype)
            params.append(prm)
    lengths = np.array([len(r) for r in rows], np.int64)
    row_ptr = np.zeros(len(rows) + 1, np.int32)
    np.cumsum(lengths, out=row_ptr[1:])
    inst = Instance(n, row_ptr, np.concatenate(rows).astype(np.int32), np.array(types, np.int8),
                    np.array(params, np.int32), name=f"planted_n{n}_s{seed}", meta={"seed": seed})
    return inst, z


def mixed_small(n: int = 64, seed: int = 0, kmax: int = 40, count: int = 160) -> Instance:
    """Small instance with every type and lengths 1..kmax (parity tests)."""
    rng = np.random.default_rng(seed)
    rows, types, params = [], [], []
    for _ in range(count):
        k = int(rng.integers(1, min(kmax, n) + 1))
        t = int(rng.integers(0, 7))
        v = rng.choice(n, size=k, replace=False)
        s = _signs(rng, k)
        prm = 0
        if t == XOR:
            prm = int(rng.integers(0, 2))
        elif t in (CARD_GE, EK):
            prm = int(rng.integers(0, k + 1))
        rows.append(((v + 1) * s).astype(np.int32))
        types.append(t)
        params.append(prm)
    lengths = np.array([len(r) for r in rows], np.int64)
    row_ptr = np.zeros(len(rows) + 1, np.int32)
    np.cumsum(lengths, out=row_ptr[1:])
    return Instance(n, row_ptr, np.concatenate(rows).astype(np.int32), np.array(types, np.int8),
                    np.array(params, np.int32), name=f"mixed_small_n{n}_s{seed}", meta={"seed": seed})


def uniform_x(rng_or_seed, R: int, n: int, near_corner: bool = False) -> np.ndarray:
    """[R][n] float32 points in [-1, 1]; near_corner draws |x| in [0.9, 1]."""
    rng = np.random.default_rng(rng_or_seed) if not isinstance(rng_or_seed, np.random.Generator) else rng_or_seed
    if near_corner:
        x = rng.uniform(0.9, 1.0, size=(R, n)) * np.where(rng.random((R, n)) < 0.5, -1, 1)
    else:
        x = rng.uniform(-1.0, 1.0, size=(R, n))
    return x.astype(np.float32)
