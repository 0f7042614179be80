"""1D hierarchical polynomial families on the master interval (0, 1).

Section 2.8.2 of the paper:

* shifted Legendre polynomials P_i by the three-term recursion
  (2.91)-(2.93), normalised so that P_i(1) = 1;
* integrated Legendre polynomials L_i = int_0^xi P_{i-1} (2.97), computed
  with the recursion (2.99)-(2.100) and completed with L_0 = 1 - xi (2.101);
* the H1 1D basis chi_i = L_i, i = 0..p, and its derivative
  chi'_0 = -1, chi'_i = P_{i-1} for i >= 1 (2.98);
* the L2 1D basis nu_i = chi'_{i+1} = P_i (2.54).

Reading taken: (2.97) prints a stray "= 0" after the integral; it is read
as the definition L_i(xi) = int_0^xi P_{i-1}(t) dt, which (2.100) confirms.

Two representations are provided: float64 evaluation at arrays of points
(used by the brute-force Gram) and exact rational coefficient lists (used by
the tests that pin this module to orthogonality, normalisation and the
integral definition).
"""
from fractions import Fraction

import numpy as np


# ----------------------------------------------------------------------------
# float64 evaluation
# ----------------------------------------------------------------------------

def legendre(nmax, x):
    """Return P[i, ...] = P_i(x) for i = 0..nmax, by (2.91)-(2.93)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((nmax + 1,) + x.shape, dtype=np.float64)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = 2.0 * x - 1.0
    t = 2.0 * x - 1.0
    for i in range(2, nmax + 1):
        out[i] = ((2 * i - 1) * t * out[i - 1] - (i - 1) * out[i - 2]) / i
    return out


def legendre_deriv(nmax, x):
    """Return dP_i/dx for i = 0..nmax, by differentiating (2.93).

    i P_i' = (2i-1) [2 P_{i-1} + (2x-1) P_{i-1}'] - (i-1) P_{i-2}'.
    Needed only where the oracle differentiates an nu factor while forming a
    full Jacobian of a vector field (those entries then cancel or are not used
    by the curl / div definitions, but the oracle does not rely on that).
    """
    x = np.asarray(x, dtype=np.float64)
    P = legendre(nmax, x)
    d = np.zeros_like(P)
    if nmax >= 1:
        d[1] = 2.0
    t = 2.0 * x - 1.0
    for i in range(2, nmax + 1):
        d[i] = ((2 * i - 1) * (2.0 * P[i - 1] + t * d[i - 1]) - (i - 1) * d[i - 2]) / i
    return d


def integrated_legendre(nmax, x):
    """Return L[i, ...] = L_i(x) for i = 0..nmax: (2.101), (2.99), (2.100)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((nmax + 1,) + x.shape, dtype=np.float64)
    out[0] = 1.0 - x
    if nmax >= 1:
        out[1] = x
    if nmax >= 2:
        P = legendre(nmax, x)
        for i in range(2, nmax + 1):
            out[i] = (P[i] - P[i - 2]) / (2.0 * (2 * i - 1))
    return out


def chi(nmax, x):
    """H1 1D basis chi_i = L_i, i = 0..nmax (Section 2.8.2)."""
    return integrated_legendre(nmax, x)


def dchi(nmax, x):
    """chi'_i: chi'_0 = -1, chi'_i = P_{i-1} (2.98), i = 0..nmax."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((nmax + 1,) + x.shape, dtype=np.float64)
    out[0] = -1.0
    if nmax >= 1:
        out[1:] = legendre(nmax - 1, x)
    return out


def ddchi(nmax, x):
    """chi''_i: 0 for i = 0, 1 and P'_{i-1} otherwise."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((nmax + 1,) + x.shape, dtype=np.float64)
    if nmax >= 2:
        out[1:] = legendre_deriv(nmax - 1, x)
    return out


def nu(nmax, x):
    """L2 1D basis nu_i = chi'_{i+1} = P_i (2.54), i = 0..nmax."""
    return legendre(nmax, x)


def dnu(nmax, x):
    return legendre_deriv(nmax, x)


# ----------------------------------------------------------------------------
# exact rational polynomials (coefficient lists, lowest degree first)
# ----------------------------------------------------------------------------

def _padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else Fraction(0)) + (b[i] if i < len(b) else Fraction(0))
            for i in range(n)]


def _pscale(a, c):
    return [c * v for v in a]


def pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            out[i + j] += u * v
    return out


def pderiv(a):
    return [i * a[i] for i in range(1, len(a))] or [Fraction(0)]


def pantideriv(a):
    """Antiderivative vanishing at 0."""
    return [Fraction(0)] + [a[i] / (i + 1) for i in range(len(a))]


def peval(a, x):
    x = Fraction(x)
    s = Fraction(0)
    for c in reversed(a):
        s = s * x + c
    return s


def pint01(a):
    """Exact integral over (0, 1)."""
    return sum(c / (i + 1) for i, c in enumerate(a))


def legendre_exact(nmax):
    """Exact P_0..P_nmax from (2.91)-(2.93)."""
    P = [[Fraction(1)]]
    if nmax >= 1:
        P.append([Fraction(-1), Fraction(2)])
    t = [Fraction(-1), Fraction(2)]
    for i in range(2, nmax + 1):
        a = _pscale(pmul(t, P[i - 1]), Fraction(2 * i - 1, i))
        b = _pscale(P[i - 2], Fraction(-(i - 1), i))
        P.append(_padd(a, b))
    return P


def integrated_legendre_exact(nmax):
    """Exact L_0..L_nmax from (2.101), (2.99), (2.100)."""
    P = legendre_exact(max(nmax, 1))
    L = [[Fraction(1), Fraction(-1)]]
    if nmax >= 1:
        L.append([Fraction(0), Fraction(1)])
    for i in range(2, nmax + 1):
        L.append(_pscale(_padd(P[i], _pscale(P[i - 2], Fraction(-1))),
                         Fraction(1, 2 * (2 * i - 1))))
    return L


def chi_exact(nmax, deriv):
    """Exact chi_i (deriv=0) or chi'_i (deriv=1), i = 0..nmax."""
    L = integrated_legendre_exact(nmax)
    if deriv == 0:
        return L
    return [pderiv(c) for c in L]
