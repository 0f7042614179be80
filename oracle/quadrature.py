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
    """Default 1D point count for a Gram of order p in `space`."""
    return p if space == "L2" else p + 1


def tensor_rule(L):
    """3D tensor rule (2.26): points xi[Q, 3] and weights w[Q], Q = L^3.

    Ordering: q = n + L*m + L*L*l for (xi_1, xi_2, xi_3) = (zeta_l, zeta_m, zeta_n).
    """
    z, w = gauss_legendre_01(L)
    l, m, n = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    xi = np.stack([z[l.ravel()], z[m.ravel()], z[n.ravel()]], axis=1)
    wq = w[l.ravel()] * w[m.ravel()] * w[n.ravel()]
    return xi, wq
