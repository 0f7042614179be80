"""Static condensation building blocks: Cholesky factor of a packed Gram and
solves with it (Section 1 and (3.7)-(3.8): eliminating s needs G^{-1} B,
G^{-1} B~ and G^{-1} l, obtained from a Cholesky factorization of G followed
by forward and backward substitution).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.

Conventions (those of LAPACK's packed 'U' routines): G = U^T U with U upper
triangular and a positive diagonal, which makes U unique.  U is stored like
G, 'U' packed column-major: (I, J), I <= J at I + J (J + 1) / 2.  The
factorization fails at the first leading minor that is not positive definite:
info = k (1-based) when the pivot of column k - 1 is not > 0, else 0.

The factor is the definition worked column by column (the up-looking order):
column j of U solves U[:j, :j]^T u = G[:j, j], and U[j, j] = sqrt(G[j, j] - u.u);
a library triangular solve is the one step taken from a library.  Everything
is FP64.
"""
import numpy as np
from scipy.linalg import solve_triangular

from .gram import packed_upper


def upper_from_packed(ap, n):
    """The upper triangle of 'U' packed storage as a full n x n array, zeros below."""
    U = np.zeros((n, n))
    off = 0
    for j in range(n):
        U[: j + 1, j] = ap[off: off + j + 1]
        off += j + 1
    return U


def cholesky_upper(G):
    """(U, info) for a symmetric G given by its upper triangle.  On failure at
    column k - 1, U holds the finished columns 0..k-2 and zeros after them."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    U = np.zeros((n, n))
    for j in range(n):
        u = solve_triangular(U[:j, :j], G[:j, j], trans="T", lower=False) if j else np.zeros(0)
        d = G[j, j] - u @ u
        if not d > 0.0:                       # NaN fails too
            return U, j + 1
        U[:j, j] = u
        U[j, j] = np.sqrt(d)
    return U, 0


def cholesky_packed(ap, n):
    """(packed U, info) from a packed 'U' Gram of dimension n."""
    U, info = cholesky_upper(upper_from_packed(np.asarray(ap, dtype=np.float64), n))
    return packed_upper(U), info


def solve_packed(up, n, B):
    """X = G^{-1} B with G = U^T U, U in packed 'U' storage; B is n x m (or n)."""
    U = upper_from_packed(np.asarray(up, dtype=np.float64), n)
    Y = solve_triangular(U, np.asarray(B, dtype=np.float64), trans="T", lower=False)   # U^T Y = B
    return solve_triangular(U, Y, lower=False)                                       # U X = Y
