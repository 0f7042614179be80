"""Pins of the adjoint-graph coupling oracle (Section 3.3, (3.17)-(3.18)),
CPU only: it does not depend on the element (the Piola maps cancel), and the
divergence theorem fixes its sum over the vertex functions of H1."""
import numpy as np
import pytest

import meshgen
from oracle import adjoint, shapes


@pytest.mark.parametrize("p", [1, 2, 3])
def test_coupling_is_the_same_on_every_element(p):
    C0 = adjoint.coupling(p)
    for e, X in enumerate(meshgen.perturbed_hexes(3, noise=0.2, seed=200 + p)):
        C = adjoint.coupling(p, "trilinear", X)
        assert np.abs(C - C0).max() <= 1e-12 * np.abs(C0).max(), e
    A = meshgen.affine_parallelepipeds(2, seed=210)
    for a in A:
        C = adjoint.coupling(p, "affine", a)
        assert np.abs(C - C0).max() <= 1e-12 * np.abs(C0).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_divergence_theorem_on_the_constant(p):
    """q = 1 is the sum of the 8 vertex functions (chi_0 + chi_1 = 1 in each
    direction), so sum_I C[I, J] = -int div v_J = -(flux of v_J out of the cube).
    For component b of V^p, v = chi_{j_b}(xi_b) prod_{d != b} nu_{j_d}(xi_d) e_b:
    chi_j(1) = [j = 1], chi_j(0) = [j = 0] and int nu_j = [j = 0], so the flux is
    ([j_b = 1] - [j_b = 0]) prod_{d != b} [j_d = 0]."""
    C = adjoint.coupling(p)
    iq = shapes.basis_index("H1", p)
    vert = np.all(iq[:, 1:] <= 1, axis=1)
    assert vert.sum() == 8
    s = C[vert].sum(axis=0)
    iv = shapes.basis_index("HDIV", p)
    expect = np.zeros(len(iv))
    for J, (b, j1, j2, j3) in enumerate(iv):
        j = (int(j1), int(j2), int(j3))
        others = all(j[d] == 0 for d in range(3) if d != b)
        expect[J] = -(int(j[b] == 1) - int(j[b] == 0)) * int(others)
    assert np.abs(s - expect).max() <= 1e-13


def test_coupling_shape():
    C = adjoint.coupling(2)
    assert C.shape == (shapes.dimension("H1", 2), shapes.dimension("HDIV", 2))


@pytest.mark.parametrize("p", [2, 3, 4])
def test_integration_by_parts_on_bubbles(p):
    """H1 functions with every index >= 2 vanish on the boundary of the cube
    (chi_i(0) = chi_i(1) = 0 for i >= 2), so int v . grad q = -int q div v."""
    A, B = adjoint.coupling_parts(p)
    iq = shapes.basis_index("H1", p)
    bub = np.all(iq[:, 1:] >= 2, axis=1)
    assert bub.any()
    scale = np.abs(B).max()
    assert np.abs(A[bub] + B[bub]).max() <= 1e-13 * scale
    assert np.abs(A[bub]).max() > 0.01 * scale            # the identity is not 0 = 0
    # and the constant has no gradient: the vertex functions' A rows sum to zero
    vert = np.all(iq[:, 1:] <= 1, axis=1)
    assert np.abs(A[vert].sum(axis=0)).max() <= 1e-13 * scale


@pytest.mark.parametrize("space,p,copies", [("H1", 2, 3), ("HDIV", 2, 3), ("HCURL", 1, 2), ("L2", 3, 3)])
def test_vector_gram_is_block_diagonal(space, p, copies):
    """(2.86), (2.88): the Gram of the product space is the scalar Gram on each
    diagonal block and zero elsewhere."""
    X = meshgen.perturbed_hexes(1, seed=230)[0]
    from oracle import gram as og
    V = og.vector_gram(space, p, "trilinear", X, copies)
    G = og.gram(space, p, "trilinear", X)
    assert np.abs(V - np.kron(np.eye(copies), G)).max() <= 1e-13 * np.abs(G).max()
