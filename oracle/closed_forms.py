"""Closed-form 1D integrals and the constant-Jacobian Kronecker form.

F^{rs}_{ij} = int_0^1 chi^<r>_i chi^<s>_j  (2.90), with chi_i = L_i, from the
chart (2.103)-(2.114) of Section 2.8.2, in exact rational arithmetic.

Readings taken:
* (2.103) gives the off-diagonal value for i = j + 2 only; j = i + 2 follows
  from the symmetry F^00_ij = F^00_ji stated with the chart.
* (2.111) states F^10 antisymmetry; it does not hold at (0, 0) and (1, 1)
  and is not used: F^10_ij = F^01_ji (2.112) is.

`kron_gram` is the Section 2.8.1 simplification (Algorithm 10 for L2)
carried to all four spaces for a constant Jacobian: each (a, b) block of the
Gram is a sum over the terms of the inner product of
coef * F^{r1 s1} (x) F^{r2 s2} (x) F^{r3 s3}, with the index shifts of the
component functions.  The term list is written here from (2.36), (2.59)-(2.60),
(2.76)-(2.77) and (2.84) independently of the brute-force module; the tests use
the two as mutual pins on affine elements.  With Fraction inputs the result
is exact.
"""
from fractions import Fraction

import numpy as np


def F00(i, j):
    if i < j:
        i, j = j, i
    # now i >= j
    if j >= 2:
        if i == j:
            return Fraction(1, 4 * (2 * j - 1) ** 2) * (Fraction(1, 2 * j + 1) + Fraction(1, 2 * j - 3))
        if i == j + 2:
            return Fraction(-1, 4 * (2 * j + 3) * (2 * j - 1) * (2 * j + 1))
        return Fraction(0)
    if j == 1:
        return {1: Fraction(1, 3), 2: Fraction(-1, 12), 3: Fraction(-1, 60)}.get(i, Fraction(0))
    # j == 0
    if i == 0:
        return Fraction(1, 3)
    if i == 1:
        return Fraction(1, 6)
    return (-1) ** i * F00(i, 1)


def F01(i, j):
    if j == 0:
        return -F01(i, 1)                                   # (2.110)
    if i == 0:                                              # (2.109)
        return {1: Fraction(1, 2), 2: Fraction(-1, 6)}.get(j, Fraction(0))
    if i == 1:                                              # (2.106)
        return {1: Fraction(1, 2), 2: Fraction(1, 6)}.get(j, Fraction(0))
    if i == 2:                                              # (2.107)
        return {1: Fraction(-1, 6), 3: Fraction(1, 30)}.get(j, Fraction(0))
    # i >= 3, j >= 1                                          (2.108)
    v = Fraction(0)
    if i == j - 1:
        v += Fraction(1, 2 * i + 1)
    if i - 1 == j:
        v -= Fraction(1, 2 * i - 3)
    return v * Fraction(1, 2 * (2 * i - 1))


def F10(i, j):
    return F01(j, i)                                        # (2.112)


def F11(i, j):
    if i >= 1 and j >= 1:
        return Fraction(1, 2 * i - 1) if i == j else Fraction(0)   # (2.113)
    if i < j:
        i, j = j, i
    # j == 0                                                  (2.114)
    return {0: Fraction(1), 1: Fraction(-1)}.get(i, Fraction(0))


_F = {(0, 0): F00, (0, 1): F01, (1, 0): F10, (1, 1): F11}


def F_table(r, s, nmax):
    """(nmax+1) x (nmax+1) object array of Fractions F^{rs}_{ij}."""
    f = _F[(r, s)]
    return np.array([[f(i, j) for j in range(nmax + 1)] for i in range(nmax + 1)], dtype=object)


# ----------------------------------------------------------------------------
# constant-Jacobian Kronecker form
# ----------------------------------------------------------------------------

def _orders(p):
    return (int(p),) * 3 if np.ndim(p) == 0 else tuple(int(x) for x in p)


def _ranges(space, p):
    q = _orders(p)
    if space == "H1":
        return [[q[d] + 1 for d in range(3)]]
    if space == "L2":
        return [[q[d] for d in range(3)]]
    if space == "HDIV":
        return [[q[d] + 1 if d == a else q[d] for d in range(3)] for a in range(3)]
    return [[q[d] if d == a else q[d] + 1 for d in range(3)] for a in range(3)]


def _shift(space, a, d):
    # index shift of the 1D factor, from (2.33), (2.54), (2.57), (2.74)
    if space == "H1":
        return 0
    if space == "L2":
        return 1
    if space == "HDIV":
        return 0 if d == a else 1
    return 1 if d == a else 0


def _inv3(J):
    a, b, c = J[0]
    d, e, f = J[1]
    g, h, k = J[2]
    det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g)
    adj = [[e * k - f * h, c * h - b * k, b * f - c * e],
           [f * g - d * k, a * k - c * g, c * d - a * f],
           [d * h - e * g, b * g - a * h, a * e - b * d]]
    return det, [[adj[i][j] / det for j in range(3)] for i in range(3)]


def block_terms(space, a, b, det, D, C, w0, w1):
    """[(coef, r[3], s[3])] of block (a, b) for constant metric data."""
    e = lambda k: [1 if d == k else 0 for d in range(3)]
    one = [1, 1, 1]
    terms = []
    if space == "H1":                                       # (2.31), (2.36), (2.44)
        terms.append((w0 * det, [0, 0, 0], [0, 0, 0]))
        for A in range(3):
            for B in range(3):
                terms.append((w1 * D[A][B] * det, e(A), e(B)))
    elif space == "L2":                                     # (2.16), (2.19)
        terms.append((w0 / det, one, one))
    elif space == "HDIV":                                   # (2.59), (2.60)
        terms.append((w0 * C[a][b] / det,
                      [1 - x for x in e(a)], [1 - x for x in e(b)]))
        terms.append((w1 / det, one, one))
    elif space == "HCURL":                                  # (2.76), (2.77), (2.84)
        terms.append((w0 * D[a][b] * det, e(a), e(b)))
        for al in (1, 2):
            for be in (1, 2):
                ca, cb = (a + al) % 3, (b + be) % 3
                sign = (-1) ** (al + be)
                terms.append((sign * w1 * C[ca][cb] / det,
                              [1 - x for x in e(ca)], [1 - x for x in e(cb)]))
    else:
        raise ValueError(space)
    return terms


def kron_gram(space, p, J, w0=1, w1=1):
    """Gram of an element with constant Jacobian J (3x3 nested lists or array);
    p is one order or three (p1, p2, p3), direction d taking its own range.

    Entries are Fractions when J, w0, w1 are Fractions/ints, floats otherwise.
    Returns an object array (exact) or float64 array.
    """
    J = [[J[i][j] for j in range(3)] for i in range(3)]
    exact = all(isinstance(x, (int, Fraction)) for row in J for x in row) and \
        isinstance(w0, (int, Fraction)) and isinstance(w1, (int, Fraction))
    if exact:
        J = [[Fraction(x) for x in row] for row in J]
        w0, w1 = Fraction(w0), Fraction(w1)
    det, Jinv = _inv3(J)
    D = [[sum(Jinv[i][k] * Jinv[j][k] for k in range(3)) for j in range(3)] for i in range(3)]
    C = [[sum(J[k][i] * J[k][j] for k in range(3)) for j in range(3)] for i in range(3)]
    R = _ranges(space, p)
    nmax = max(_orders(p)) + 1
    Ft = {rs: F_table(rs[0], rs[1], nmax) for rs in _F}
    if not exact:
        Ft = {k: v.astype(np.float64) for k, v in Ft.items()}
    offs = np.cumsum([0] + [int(np.prod(r)) for r in R])
    n = int(offs[-1])
    G = np.zeros((n, n), dtype=object if exact else np.float64)
    if exact:
        G[:, :] = Fraction(0)
    for a in range(len(R)):
        for b in range(len(R)):
            blk = None
            for coef, r, s in block_terms(space, a, b, det, D, C, w0, w1):
                facs = []
                for d in range(3):
                    ia = np.arange(R[a][d]) + _shift(space, a, d)
                    jb = np.arange(R[b][d]) + _shift(space, b, d)
                    facs.append(Ft[(r[d], s[d])][np.ix_(ia, jb)])
                term = np.kron(facs[2], np.kron(facs[1], facs[0])) * coef
                blk = term if blk is None else blk + term
            G[offs[a]:offs[a + 1], offs[b]:offs[b + 1]] = blk
    return G
