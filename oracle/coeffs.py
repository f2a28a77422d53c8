"""Exact spectra and Walsh-Fourier coefficients of symmetric constraints.

TEST INFRASTRUCTURE. This module belongs to the correctness oracle: only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import it.
It shares no code with the HIP path.

Conventions (Background, "Walsh-Fourier Transformation"): Boolean True maps to
-1 and False to +1.  A symmetric constraint over k literals is described by its
spectrum sp[t], t = 0..k, where sp[t] = -1 when the constraint holds with exactly
t true literals and +1 otherwise.  The coefficients a_j = f_hat(S) for |S| = j
follow the general formula of eq. (wfcoef):

    a_0 = 2^-k * sum_t C(k, t) sp_t
    a_j = [rho^(j-1)] g(rho) / (C(k-1, j-1) 2^(k-1)),   j >= 1
    g(rho) = sum_{i=0}^{k-1} d_i C(k-1, i) (1+rho)^(k-1-i) (1-rho)^i
    d_i = (sp_i - sp_{i+1}) / 2

Everything here is exact (Python integers and Fractions).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb

# Constraint type codes (Background, "Pseudo-Boolean Representation"; Table 2).
OR = 0       # at least one literal true
XOR = 1      # parity: number of true literals = param (mod 2); param 1 is the paper's XOR
CARD_GE = 2  # at least param literals true
NAE = 3      # not all equal: 0 < #true < k
EO = 4       # exactly one true
AMO = 5      # at most one true
EK = 6       # exactly param true

TYPE_NAMES = {OR: "OR", XOR: "XOR", CARD_GE: "CARD_GE", NAE: "NAE", EO: "EO", AMO: "AMO", EK: "EK"}


def holds(ctype: int, k: int, param: int, t: int) -> bool:
    """Whether a constraint of the given type holds with exactly t of k literals true."""
    if ctype == OR:
        return t >= 1
    if ctype == XOR:
        return t % 2 == param
    if ctype == CARD_GE:
        return t >= param
    if ctype == NAE:
        return 0 < t < k
    if ctype == EO:
        return t == 1
    if ctype == AMO:
        return t <= 1
    if ctype == EK:
        return t == param
    raise ValueError(f"unknown constraint type {ctype}")


def spectrum(ctype: int, k: int, param: int = 0) -> tuple[int, ...]:
    """sp_t for t = 0..k (eq. wfcoef: -1 where the constraint holds, +1 elsewhere)."""
    if k < 1:
        raise ValueError("constraint needs at least one literal")
    return tuple(-1 if holds(ctype, k, param, t) else 1 for t in range(k + 1))


def _times_one_minus_over_one_plus(poly: list[int]) -> list[int]:
    """Exact p(rho) * (1 - rho) / (1 + rho) for a polynomial divisible by (1 + rho)."""
    # divide by (1 + rho): p = q (1 + rho)  =>  q_j = p_j - q_{j-1}
    q = []
    prev = 0
    for j in range(len(poly) - 1):
        prev = poly[j] - prev
        q.append(prev)
    if poly[-1] - prev != 0:
        raise ArithmeticError("polynomial not divisible by (1 + rho)")
    # multiply by (1 - rho)
    out = [0] * len(poly)
    for j, c in enumerate(q):
        out[j] += c
        out[j + 1] -= c
    return out


def g_polynomial(sp: tuple[int, ...]) -> list[int]:
    """Integer coefficients of g(rho) from eq. (wfcoef), lowest degree first.

    The terms (1+rho)^(k-1-i) (1-rho)^i are generated one from the previous by
    multiplying with (1-rho)/(1+rho), which keeps every step exact.
    """
    k = len(sp) - 1
    d = [(sp[i] - sp[i + 1]) // 2 for i in range(k)]
    term = [comb(k - 1, j) for j in range(k)]  # (1+rho)^(k-1)
    g = [0] * k
    for i in range(k):
        if d[i] != 0:
            scale = d[i] * comb(k - 1, i)
            for j in range(k):
                g[j] += scale * term[j]
        if i + 1 < k:
            term = _times_one_minus_over_one_plus(term)
    return g


@lru_cache(maxsize=None)
def wf_coefficients(sp: tuple[int, ...]) -> tuple[Fraction, ...]:
    """a_j = f_hat(S), |S| = j, for j = 0..k, from eq. (wfcoef)."""
    k = len(sp) - 1
    a0 = Fraction(sum(comb(k, t) * sp[t] for t in range(k + 1)), 2 ** k)
    g = g_polynomial(sp)
    rest = [Fraction(g[j - 1], comb(k - 1, j - 1) * 2 ** (k - 1)) for j in range(1, k + 1)]
    return (a0, *rest)


def wf_coefficients_f64(sp: tuple[int, ...]) -> list[float]:
    """The exact coefficients rounded once to the nearest float64."""
    return [float(c) for c in wf_coefficients(tuple(sp))]


def d_spectrum(sp: tuple[int, ...]) -> list[int]:
    """Discrete derivative d_i = (sp_i - sp_{i+1}) / 2, i = 0..k-1 (eq. wfcoef)."""
    return [(sp[i] - sp[i + 1]) // 2 for i in range(len(sp) - 1)]
