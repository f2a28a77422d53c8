"""Pins of the oracle's exact coefficients (eq. wfcoef) against independent facts.

- the Walsh transform by its definition, f_hat(S) = 2^-k sum_z f(z) prod_{i in S} z_i,
  enumerated over all 2^k corners for k <= 10;
- the closed forms of Appendix A (OR, EO, EK, AMO, NAE, XOR, CARD);
- the corner property FE(z) = sp_{#true(z)} of the resulting polynomial.
"""
from fractions import Fraction
from itertools import product
from math import comb

import pytest

from oracle import coeffs as C

ALL_TYPES = [C.OR, C.XOR, C.CARD_GE, C.NAE, C.EO, C.AMO, C.EK]


def params_for(ctype, k):
    if ctype == C.XOR:
        return [0, 1]
    if ctype in (C.CARD_GE, C.EK):
        return list(range(0, k + 1))
    return [0]


def brute_walsh(sp):
    """f_hat(S) for S = the first j coordinates, j = 0..k, from the definition."""
    k = len(sp) - 1
    out = []
    for j in range(k + 1):
        acc = 0
        for z in product((1, -1), repeat=k):
            t = sum(1 for zi in z if zi == -1)
            chi = 1
            for i in range(j):
                chi *= z[i]
            acc += sp[t] * chi
        out.append(Fraction(acc, 2 ** k))
    return out


@pytest.mark.parametrize("k", range(1, 11))
def test_general_formula_matches_brute_force_walsh(k):
    for ctype in ALL_TYPES:
        for prm in params_for(ctype, k):
            sp = C.spectrum(ctype, k, prm)
            assert list(C.wf_coefficients(sp)) == brute_walsh(sp), (ctype, k, prm)


def test_brute_force_symmetry_assumption():
    # the coefficient depends only on |S|: check every S for one asymmetric-looking case
    sp = C.spectrum(C.CARD_GE, 5, 2)
    k = 5
    a = C.wf_coefficients(sp)
    for S in product((0, 1), repeat=k):
        acc = 0
        for z in product((1, -1), repeat=k):
            t = sum(1 for zi in z if zi == -1)
            chi = 1
            for i in range(k):
                if S[i]:
                    chi *= z[i]
            acc += sp[t] * chi
        assert Fraction(acc, 2 ** k) == a[sum(S)]


# ---------------------------------------------------------------- Appendix A

def poly_coeff(poly_factors, deg):
    """[rho^deg] of a product of (c0 + c1 rho)^e factors given as (c0, c1, e)."""
    poly = [Fraction(1)]
    for c0, c1, e in poly_factors:
        for _ in range(e):
            nxt = [Fraction(0)] * (len(poly) + 1)
            for i, v in enumerate(poly):
                nxt[i] += c0 * v
                nxt[i + 1] += c1 * v
            poly = nxt
    return poly[deg] if deg < len(poly) else Fraction(0)


@pytest.mark.parametrize("n", range(1, 25))
def test_appendix_a_or(n):
    a = C.wf_coefficients(C.spectrum(C.OR, n))
    assert a[0] == Fraction(1, 2 ** (n - 1)) - 1
    assert all(v == Fraction(1, 2 ** (n - 1)) for v in a[1:])


@pytest.mark.parametrize("n", range(1, 25))
def test_appendix_a_eo(n):
    a = C.wf_coefficients(C.spectrum(C.EO, n))
    assert a[0] == 1 - Fraction(n, 2 ** (n - 1))
    for s in range(1, n + 1):
        assert a[s] == Fraction(2 * s - n, 2 ** (n - 1))


@pytest.mark.parametrize("n", range(2, 25))
def test_appendix_a_amo_with_corrected_constant(n):
    """AMO: the |S| != 0 coefficients are as printed; the constant term is
    1 - (n+1)/2^(n-1) (the printed (n-1) does not match the definition)."""
    a = C.wf_coefficients(C.spectrum(C.AMO, n))
    for s in range(1, n + 1):
        assert a[s] == Fraction(2 * s - n - 1, 2 ** (n - 1))
    assert a[0] == 1 - Fraction(n + 1, 2 ** (n - 1))
    # the printed constant disagrees with the brute-force transform
    if n <= 10:
        assert brute_walsh(C.spectrum(C.AMO, n))[0] != 1 - Fraction(n - 1, 2 ** (n - 1))


@pytest.mark.parametrize("n", range(2, 25))
def test_appendix_a_nae(n):
    a = C.wf_coefficients(C.spectrum(C.NAE, n))
    assert a[0] == Fraction(1, 2 ** (n - 2)) - 1
    for s in range(1, n + 1):
        assert a[s] == (Fraction(1, 2 ** (n - 2)) if s % 2 == 0 else 0)


@pytest.mark.parametrize("n", range(1, 25))
def test_appendix_a_xor(n):
    a = C.wf_coefficients(C.spectrum(C.XOR, n, 1))
    assert a[n] == 1
    assert all(v == 0 for v in a[:n])


@pytest.mark.parametrize("n", range(1, 16))
def test_appendix_a_card(n):
    for kap in range(1, n + 1):
        a = C.wf_coefficients(C.spectrum(C.CARD_GE, n, kap))
        assert a[0] == 1 - Fraction(sum(comb(n, i) for i in range(kap, n + 1)), 2 ** (n - 1))
        for s in range(1, n + 1):
            g = poly_coeff([(1, 1, n - kap), (1, -1, kap - 1)], s - 1)
            assert a[s] == comb(n - 1, kap - 1) * g / (comb(n - 1, s - 1) * 2 ** (n - 1)), (n, kap, s)


@pytest.mark.parametrize("n", range(2, 16))
def test_appendix_a_ek(n):
    """EK with (1 - rho) in place of the printed (1 - p); valid for 1 <= k < n."""
    for kap in range(1, n):
        a = C.wf_coefficients(C.spectrum(C.EK, n, kap))
        assert a[0] == 1 - Fraction(comb(n, kap), 2 ** (n - 1))
        for s in range(1, n + 1):
            # g_EK = ((2k - n) + n rho)/k * C(n-1, k-1) (1+rho)^(n-k-1) (1-rho)^(k-1)
            base = [(1, 1, n - kap - 1), (1, -1, kap - 1)]
            g = (2 * kap - n) * poly_coeff(base, s - 1) + n * (poly_coeff(base, s - 2) if s >= 2 else 0)
            g = g * Fraction(comb(n - 1, kap - 1), kap)
            assert a[s] == g / (comb(n - 1, s - 1) * 2 ** (n - 1)), (n, kap, s)
            # the second printed form of g_EK agrees
            g2 = Fraction(comb(n, kap), n) * ((2 * kap - n) * poly_coeff(base, s - 1)
                                              + n * (poly_coeff(base, s - 2) if s >= 2 else 0))
            assert g == g2


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 12])
def test_polynomial_takes_spectrum_at_corners(k):
    """sum_j a_j e_j(z) = sp_{#true(z)} at every corner (exact arithmetic)."""
    for ctype in ALL_TYPES:
        for prm in params_for(ctype, k):
            sp = C.spectrum(ctype, k, prm)
            a = C.wf_coefficients(sp)
            for z in product((1, -1), repeat=k):
                e = [1] + [0] * k
                for zi in z:
                    for j in range(k, 0, -1):
                        e[j] += zi * e[j - 1]
                t = sum(1 for zi in z if zi == -1)
                assert sum(a[j] * e[j] for j in range(k + 1)) == sp[t]


def test_long_coefficients_exact_and_bounded():
    # k = 256 classes finish and satisfy sum_j C(k,j) a_j^2 = 1 (Parseval: f is +/-1 valued)
    for ctype, prm in [(C.OR, 0), (C.XOR, 1), (C.CARD_GE, 128), (C.NAE, 0)]:
        sp = C.spectrum(ctype, 256, prm)
        a = C.wf_coefficients(sp)
        assert sum(comb(256, j) * a[j] ** 2 for j in range(257)) == 1


def test_spectrum_conventions():
    assert C.spectrum(C.OR, 3) == (1, -1, -1, -1)
    assert C.spectrum(C.XOR, 3, 1) == (1, -1, 1, -1)
    assert C.spectrum(C.CARD_GE, 4, 0) == (-1, -1, -1, -1, -1)
    assert C.spectrum(C.NAE, 3) == (1, -1, -1, 1)
    assert C.spectrum(C.EK, 3, 3) == (1, 1, 1, -1)
