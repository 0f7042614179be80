"""Coupling block of the adjoint graph inner product (Section 3.3).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.

The ultraweak acoustics formulation tests with (q, v) in H1 x H(div), and its
adjoint graph inner product (3.17) couples the two spaces through

    (v, grad q)_K - (div v, q)_K,

the real integral that (3.18) multiplies by i omega (the Hermitian counterpart
is its transpose).  This module computes, for one element K,

    C[I, J] = int_K ( v_J . grad q_I - q_I div v_J ) dx,   q_I in W^p, v_J in V^p,

by brute force: the physical fields of the two spaces (their Piola maps, as in
gram.physical_fields) at the tensor Gauss-Legendre points, weighted by w |J|.
After the Piola maps the integrand is the master-element polynomial
v_hat . grad_hat q_hat - q_hat div_hat v_hat of degree <= 2p per direction, so
the (p+1)-point rule is exact and C does not depend on K (checked by the
tests, not assumed here).  The other terms of (3.17) are the H1 and H(div)
Grams with w0 = omega^2 + alpha and w1 = 1.
"""
import numpy as np

from . import geometry, gram, quadrature


def unit_cube():
    """The reference cube as a trilinear element, [8, 3]."""
    return geometry.corner_bits().astype(np.float64)


def coupling_parts(p, kind="trilinear", geom=None, L=None):
    """(A, B) with A[I, J] = int_K v_J . grad q_I and B[I, J] = int_K q_I div v_J,
    [n_H1, n_Hdiv] each, for one element (default: the reference cube)."""
    if geom is None:
        kind, geom = "trilinear", unit_cube()
    xi, wq = quadrature.tensor_rule(p + 1 if L is None else L)
    fq, gq, detJ = gram.physical_fields("H1", p, kind, geom, xi)     # q, grad q
    fv, gv, _ = gram.physical_fields("HDIV", p, kind, geom, xi)      # v, div v
    W = wq * detJ
    A = np.zeros((fq.shape[1], fv.shape[1]))
    for c in range(3):
        A += (gq[:, :, c] * W[:, None]).T @ fv[:, :, c]
    B = (fq[:, :, 0] * W[:, None]).T @ gv[:, :, 0]
    return A, B


def coupling(p, kind="trilinear", geom=None, L=None):
    """C = A - B, [n_H1, n_Hdiv], float64."""
    A, B = coupling_parts(p, kind, geom, L)
    return A - B
