"""Pins of the oracle's 1D layer against facts fixed by the paper and by
mathematics (not by retyping the oracle's own formulas).

* Legendre: orthogonality with norm 1/(2i+1) (2.95), average zero (2.96),
  P_i(1) = 1 (text after (2.93)), parity about 1/2 (Section 2.8.2).  These
  determine the shifted Legendre family uniquely.
* Integrated Legendre: the integral definition (2.97), the bubble property
  L_i(0) = L_i(1) = 0 for i >= 2, L_0 + L_1 = 1 (2.101).
* Gauss-Legendre: exactness for degree <= 2L - 1 (text after (2.22)).
* The chart (2.103)-(2.114): equal to exact integration of the products.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import closed_forms, poly1d, quadrature

NMAX = 12


def test_legendre_orthogonality_and_normalisation_exact():
    P = poly1d.legendre_exact(NMAX)
    for i in range(NMAX + 1):
        assert len(P[i]) == i + 1 and P[i][-1] != 0          # degree exactly i
        assert poly1d.peval(P[i], 1) == 1                       # P_i(1) = 1
        assert poly1d.peval(P[i], 0) == (-1) ** i               # parity about 1/2
        for j in range(NMAX + 1):
            v = poly1d.pint01(poly1d.pmul(P[i], P[j]))
            assert v == (Fraction(1, 2 * i + 1) if i == j else 0)
        if i >= 1:
            assert poly1d.pint01(P[i]) == 0                     # (2.96)


def test_legendre_parity_about_half():
    x = np.linspace(0.0, 1.0, 17)
    P = poly1d.legendre(NMAX, x)
    Pm = poly1d.legendre(NMAX, 1.0 - x)
    for i in range(NMAX + 1):
        np.testing.assert_allclose(Pm[i], (-1) ** i * P[i], atol=1e-13)


def test_integrated_legendre_integral_definition_exact():
    P = poly1d.legendre_exact(NMAX)
    L = poly1d.integrated_legendre_exact(NMAX)
    assert poly1d._padd(L[0], L[1]) == [Fraction(1), Fraction(0)]   # L0 + L1 = 1
    for i in range(1, NMAX + 1):
        ref = poly1d.pantideriv(P[i - 1])                       # (2.97)
        a = L[i] + [Fraction(0)] * (len(ref) - len(L[i]))
        b = ref + [Fraction(0)] * (len(L[i]) - len(ref))
        assert a == b, i
        if i >= 2:
            assert poly1d.peval(L[i], 0) == 0 and poly1d.peval(L[i], 1) == 0


def test_float_families_match_exact():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, 9)
    P = poly1d.legendre_exact(NMAX)
    L = poly1d.integrated_legendre_exact(NMAX)
    dP = [poly1d.pderiv(c) for c in P]
    fP, fdP = poly1d.legendre(NMAX, x), poly1d.legendre_deriv(NMAX, x)
    fchi, fdchi, fddchi = poly1d.chi(NMAX, x), poly1d.dchi(NMAX, x), poly1d.ddchi(NMAX, x)
    for k in range(NMAX + 1):
        for t, xv in enumerate(x):
            fx = Fraction(float(xv))
            assert abs(fP[k, t] - float(poly1d.peval(P[k], fx))) < 1e-13
            assert abs(fdP[k, t] - float(poly1d.peval(dP[k], fx))) < 1e-11
            assert abs(fchi[k, t] - float(poly1d.peval(L[k], fx))) < 1e-14
            dL = poly1d.pderiv(L[k])
            assert abs(fdchi[k, t] - float(poly1d.peval(dL, fx))) < 1e-13
            assert abs(fddchi[k, t] - float(poly1d.peval(poly1d.pderiv(dL), fx))) < 1e-11


@pytest.mark.parametrize("L", range(1, 14))
def test_gauss_legendre_exactness(L):
    z, w = quadrature.gauss_legendre_01(L)
    assert np.all((z > 0) & (z < 1))
    assert abs(w.sum() - 1.0) < 1e-14
    for k in range(2 * L):
        assert abs(np.dot(w, z ** k) * (k + 1) - 1.0) < 1e-14
    # degree 2L: the Gauss-Legendre error constant on (0, 1),
    # int - sum = f^(2L) (L!)^4 / ((2L+1) ((2L)!)^3) with f = xi^(2L)
    if L <= 8:
        from math import factorial
        E = factorial(L) ** 4 / ((2 * L + 1) * factorial(2 * L) ** 2)
        err = 1.0 / (2 * L + 1) - np.dot(w, z ** (2 * L))
        assert abs(err / E - 1.0) < 1e-6


def test_closed_form_chart_equals_exact_integrals():
    for r in (0, 1):
        for s in (0, 1):
            A = poly1d.chi_exact(NMAX, r)
            B = poly1d.chi_exact(NMAX, s)
            tab = closed_forms.F_table(r, s, NMAX)
            for i in range(NMAX + 1):
                for j in range(NMAX + 1):
                    assert tab[i, j] == poly1d.pint01(poly1d.pmul(A[i], B[j])), (r, s, i, j)


def test_chart_matches_float_quadrature():
    z, w = quadrature.gauss_legendre_01(NMAX + 2)
    T = [poly1d.chi(NMAX, z), poly1d.dchi(NMAX, z)]
    for r in (0, 1):
        for s in (0, 1):
            num = np.einsum("l,il,jl->ij", w, T[r], T[s])
            ref = closed_forms.F_table(r, s, NMAX).astype(float)
            np.testing.assert_allclose(num, ref, atol=2e-15)
