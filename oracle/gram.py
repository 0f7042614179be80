"""Brute-force Gram matrices: the conventional algorithm family.

For an element K with map x_K, every entry is the quadrature sum (2.26)

    G_IJ = sum_{l,m,n} w_l w_m w_n |J| ( w0 <f_I, f_J> + w1 <g_I, g_J> )

over the L^3 tensor Gauss-Legendre points, where f_I is the physical shape
function (the Piola image of the master function, (2.3)-(2.6)) and g_I its
physical grad / curl / div:

* H1      f = u_hat,               g = J^{-T} grad_hat u_hat          (2.28), (2.31)
* H(curl) f = J^{-T} E_hat,        g = |J|^{-1} J curl_hat E_hat      (2.65), (2.68)
* H(div)  f = |J|^{-1} J V_hat,    g = |J|^{-1} div_hat V_hat         (2.46), (2.49)
* L2      f = |J|^{-1} q_hat,      (no derivative part)               (2.14), (2.16)

The commuting relations used for g are the ones stated in Sections 2.4-2.6.
w0 and w1 weight the value and derivative parts; w0 = w1 = 1 are the
paper's inner products.  The only library primitive used beyond element-wise
numpy is a matrix product for the sum over points.  Costs are O(L^3 n^2).

Readings taken: the default number of points follows Algorithms 2, 5, 7, 9
(L = p for L2, p + 1 otherwise).  For non-affine maps the integrand is
rational, so the result depends on L; comparisons are made at equal L.
det J must be positive at every point (the map is a diffeomorphism,
Section 2.2); `jacobian_ok` reports it.
"""
import numpy as np

from . import geometry, quadrature, shapes

# Levi-Civita symbol: (curl F)_c = sum_{e,k} eps[c, e, k] d_e F_k, the
# component form of (2.67).
_EPS = np.zeros((3, 3, 3))
for _c, _e, _k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    _EPS[_c, _e, _k] = 1.0
    _EPS[_c, _k, _e] = -1.0


def _rule(space, p, L):
    if L is None:
        L = quadrature.default_points(space, p)
    return quadrature.tensor_rule(L)


def physical_fields(space, p, kind, geom, xi, subset=None):
    """Return (f[Q, n, c], g[Q, n, c'] or None, detJ[Q]) at points xi."""
    J = geometry.jacobian(kind, geom, xi)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    comp, val, grad = shapes.evaluate(space, p, xi, subset)
    if space == "H1":
        f = val[:, :, None]
        g = np.einsum("qji,qnj->qni", Jinv, grad)
        return f, g, detJ
    if space == "L2":
        f = (val / detJ[:, None])[:, :, None]
        return f, None, detJ
    if space == "HDIV":
        cols = J[:, :, comp]                       # [Q, 3, n]: J e_a
        f = np.transpose(cols, (0, 2, 1)) * (val / detJ[:, None])[:, :, None]
        n = comp.shape[0]
        divhat = grad[:, np.arange(n), comp]       # d_a of component a
        g = (divhat / detJ[:, None])[:, :, None]
        return f, g, detJ
    if space == "HCURL":
        rows = Jinv[:, comp, :]                    # [Q, n, 3]: (J^{-T} e_a)_i = Jinv[a, i]
        f = rows * val[:, :, None]
        eps_a = _EPS[:, :, comp]                   # [3 (c), 3 (e), n]
        curlhat = np.einsum("cen,qne->qnc", eps_a, grad)
        g = np.einsum("qij,qnj->qni", J, curlhat) / detJ[:, None, None]
        return f, g, detJ
    raise ValueError(space)


def jacobian_ok(space, p, kind, geom, L=None):
    xi, _ = _rule(space, p, L)
    J = geometry.jacobian(kind, geom, xi)
    return bool(np.all(np.linalg.det(J) > 0.0))


def gram(space, p, kind, geom, L=None, w0=1.0, w1=1.0):
    """Full n x n Gram matrix of one element (float64)."""
    xi, wq = _rule(space, p, L)
    f, g, detJ = physical_fields(space, p, kind, geom, xi)
    W = wq * detJ
    G = np.zeros((f.shape[1], f.shape[1]))
    for c in range(f.shape[2]):
        G += w0 * ((f[:, :, c] * W[:, None]).T @ f[:, :, c])
    if g is not None and w1 != 0.0:
        for c in range(g.shape[2]):
            G += w1 * ((g[:, :, c] * W[:, None]).T @ g[:, :, c])
    return G


def vector_gram(space, p, kind, geom, copies, L=None, w0=1.0, w1=1.0):
    """Gram of the `copies`-fold product of a space (Section 2.7): basis
    functions e_k (x) f_I, k < copies, ordered copy by copy, with the Frobenius
    inner products of (2.85) and (2.87), (div Theta_I)^T (div Theta_J) for the
    derivative part.  Built from the matrix-valued fields directly, without the
    block structure that (2.86) and (2.88) derive."""
    xi, wq = _rule(space, p, L)
    f, g, detJ = physical_fields(space, p, kind, geom, xi)
    W = wq * detJ
    Q, n = f.shape[0], f.shape[1]

    def lift(h):
        out = np.zeros((Q, copies * n, copies * h.shape[2]))
        for k in range(copies):
            out[:, k * n:(k + 1) * n, k * h.shape[2]:(k + 1) * h.shape[2]] = h
        return out

    F = lift(f)
    G = np.zeros((copies * n, copies * n))
    for c in range(F.shape[2]):
        G += w0 * ((F[:, :, c] * W[:, None]).T @ F[:, :, c])
    if g is not None and w1 != 0.0:
        Gd = lift(g)
        for c in range(Gd.shape[2]):
            G += w1 * ((Gd[:, :, c] * W[:, None]).T @ Gd[:, :, c])
    return G


def gram_entries(space, p, kind, geom, I, J, L=None, w0=1.0, w1=1.0):
    """G_IJ for the index lists I, J (same length), computed entry by entry."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    need = np.unique(np.concatenate([I, J]))
    pos = {int(k): t for t, k in enumerate(need)}
    xi, wq = _rule(space, p, L)
    f, g, detJ = physical_fields(space, p, kind, geom, xi, subset=need)
    W = wq * detJ
    ii = np.array([pos[int(k)] for k in I])
    jj = np.array([pos[int(k)] for k in J])
    out = w0 * np.einsum("q,qnc,qnc->n", W, f[:, ii, :], f[:, jj, :])
    if g is not None and w1 != 0.0:
        out = out + w1 * np.einsum("q,qnc,qnc->n", W, g[:, ii, :], g[:, jj, :])
    return out


def gram_matvec(space, p, kind, geom, r, L=None, w0=1.0, w1=1.0):
    """G @ r in O(L^3 n) without forming G (a Freivalds-style probe)."""
    xi, wq = _rule(space, p, L)
    f, g, detJ = physical_fields(space, p, kind, geom, xi)
    W = wq * detJ
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros(f.shape[1])
    for c in range(f.shape[2]):
        out += w0 * (f[:, :, c].T @ (W * (f[:, :, c] @ r)))
    if g is not None and w1 != 0.0:
        for c in range(g.shape[2]):
            out += w1 * (g[:, :, c].T @ (W * (g[:, :, c] @ r)))
    return out


def packed_upper(G):
    """LAPACK 'U' packed column-major storage: (I, J), I <= J at I + J(J+1)/2."""
    n = G.shape[0]
    return np.concatenate([G[: j + 1, j] for j in range(n)])


def unpack_upper(ap, n):
    """Inverse of packed_upper: symmetric n x n matrix from 'U' packed storage."""
    G = np.zeros((n, n))
    off = 0
    for j in range(n):
        G[: j + 1, j] = ap[off: off + j + 1]
        off += j + 1
    return G + np.triu(G, 1).T


def packed_offset(I, J):
    """Offset of (I, J), I <= J, in 'U' packed storage."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    return I + J * (J + 1) // 2
