"""Element maps x_K: (0,1)^3 -> K and their Jacobians (2.2).

Two kinds of map, each given by plain float64 data per element:

* trilinear: 8 vertices X[v, 3], vertex v = v1 + 2 v2 + 4 v3 sits at the
  master corner (v1, v2, v3); x(xi) = sum_v X_v prod_d (xi_d if v_d else 1 - xi_d).
* affine: 12 numbers, x0[3] followed by J[3, 3] row-major, x(xi) = x0 + J xi,
  J_ij = d x_i / d xi_j.

The paper fixes neither a vertex ordering nor an input format; these are the
readings used throughout the repository.  The paper assumes x_K is a
diffeomorphism (Section 2.2); an element with det J <= 0 at a quadrature
point is reported as invalid.
"""
import numpy as np


def corner_bits():
    v = np.arange(8)
    return np.stack([v & 1, (v >> 1) & 1, (v >> 2) & 1], axis=1)


def trilinear_map(X, xi):
    """x(xi) for vertices X[8, 3] at points xi[Q, 3]."""
    X = np.asarray(X, dtype=np.float64).reshape(8, 3)
    bits = corner_bits()
    xi = np.asarray(xi, dtype=np.float64)
    phi = np.ones((xi.shape[0], 8))
    for d in range(3):
        f = np.where(bits[None, :, d] == 1, xi[:, d:d + 1], 1.0 - xi[:, d:d + 1])
        phi *= f
    return phi @ X


def trilinear_jacobian(X, xi):
    """J[Q, 3, 3] with J[q, i, j] = d x_i / d xi_j at xi[q]."""
    X = np.asarray(X, dtype=np.float64).reshape(8, 3)
    bits = corner_bits()
    xi = np.asarray(xi, dtype=np.float64)
    Q = xi.shape[0]
    J = np.zeros((Q, 3, 3))
    for j in range(3):
        dphi = np.ones((Q, 8))
        for d in range(3):
            if d == j:
                f = np.where(bits[None, :, d] == 1, 1.0, -1.0) * np.ones((Q, 1))
            else:
                f = np.where(bits[None, :, d] == 1, xi[:, d:d + 1], 1.0 - xi[:, d:d + 1])
            dphi = dphi * f
        J[:, :, j] = dphi @ X
    return J


def affine_parts(A):
    A = np.asarray(A, dtype=np.float64).reshape(12)
    return A[:3].copy(), A[3:].reshape(3, 3).copy()


def affine_jacobian(A, xi):
    _, J = affine_parts(A)
    Q = np.asarray(xi).shape[0]
    return np.broadcast_to(J, (Q, 3, 3)).copy()


def jacobian(kind, geom, xi):
    if kind == "trilinear":
        return trilinear_jacobian(geom, xi)
    if kind == "affine":
        return affine_jacobian(geom, xi)
    raise ValueError(kind)


def map_points(kind, geom, xi):
    if kind == "trilinear":
        return trilinear_map(geom, xi)
    x0, J = affine_parts(geom)
    return x0[None, :] + np.asarray(xi) @ J.T
