"""Gauss-Legendre quadrature on (0, 1).

The paper integrates every 1D factor with an N-point rule exact for
polynomials of degree 2N-1 (text after (2.22)), the same rule in all three
directions (text after (2.25)), and the 3D rule is its tensor product
(2.26).  That rule is Gauss-Legendre; the oracle takes it from numpy's
library routine on (-1, 1) and maps it affinely to (0, 1).

Default number of points (reading of Algorithms 2, 5, 7, 9): L = p + 1 for
H1, H(curl), H(div) and L = p for L2.
"""
import numpy as np


def gauss_legendre_01(L):
    """Return (zeta[L], w[L]) of the L-point Gauss-Legendre rule on (0, 1)."""
    if L < 1:
        raise ValueError("need at least one quadrature point")
    x, w = np.polynomial.legendre.leggauss(L)
    return 0.5 * (x + 1.0), 0.5 * w


def default_points(space, p):
    """Default 1D point count for a Gram of order p in `space`; for orders
    given per direction, the count of each direction from its own order (one
    rule per coordinate, the option the text after Algorithm 2 allows)."""
    if np.ndim(p) != 0:
        return tuple(default_points(space, int(x)) for x in p)
    return p if space == "L2" else p + 1


def tensor_rule(L):
    """3D tensor rule (2.26): points xi[Q, 3] and weights w[Q], Q = L1 L2 L3
    (L an int: the same rule in every direction, or a triple).

    Ordering: q = n + L3*m + L3*L2*l for (xi_1, xi_2, xi_3) = (zeta_l, zeta_m, zeta_n).
    """
    L1, L2, L3 = (L,) * 3 if np.ndim(L) == 0 else tuple(int(x) for x in L)
    (z1, w1), (z2, w2), (z3, w3) = gauss_legendre_01(L1), gauss_legendre_01(L2), gauss_legendre_01(L3)
    l, m, n = np.meshgrid(np.arange(L1), np.arange(L2), np.arange(L3), indexing="ij")
    xi = np.stack([z1[l.ravel()], z2[m.ravel()], z3[n.ravel()]], axis=1)
    wq = w1[l.ravel()] * w2[m.ravel()] * w3[n.ravel()]
    return xi, wq
