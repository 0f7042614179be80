"""Pins of the oracle at non-uniform orders (p1, p2, p3) (the text after
Algorithm 2: one 1D rule per coordinate), CPU only.  The quadrature oracle
against the exact Kronecker form of constant-Jacobian elements, which takes
its 1D integrals from the closed-form chart (2.103)-(2.114); the dimensions
against their product formulas; per-direction rules against one larger rule."""
from fractions import Fraction

import numpy as np
import pytest

import meshgen
from oracle import closed_forms, quadrature, shapes
from oracle import gram as og

SPACES = ["H1", "HCURL", "HDIV", "L2"]
TUPLES = [(1, 2, 3), (3, 1, 2), (2, 4, 1), (4, 2, 3)]


@pytest.mark.parametrize("q", TUPLES)
def test_dimensions(q):
    p1, p2, p3 = q
    assert shapes.dimension("H1", q) == (p1 + 1) * (p2 + 1) * (p3 + 1)
    assert shapes.dimension("L2", q) == p1 * p2 * p3
    assert shapes.dimension("HDIV", q) == (p1 + 1) * p2 * p3 + p1 * (p2 + 1) * p3 + p1 * p2 * (p3 + 1)
    assert shapes.dimension("HCURL", q) == p1 * (p2 + 1) * (p3 + 1) + (p1 + 1) * p2 * (p3 + 1) + (p1 + 1) * (p2 + 1) * p3
    # exact sequence: dim W - dim Q + dim V - dim Y = 1 (the Euler characteristic of the cube)
    assert (shapes.dimension("H1", q) - shapes.dimension("HCURL", q) + shapes.dimension("HDIV", q)
            - shapes.dimension("L2", q)) == 1


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("q", TUPLES)
def test_affine_matches_kronecker_form(space, q):
    """Constant Jacobian: the per-direction Gauss rules are exact, so the
    quadrature oracle equals the Kronecker form built from exact 1D integrals."""
    A = meshgen.affine_parallelepipeds(1, seed=500 + sum(q))[0]
    J = A[3:].reshape(3, 3)
    G = og.gram(space, q, "affine", A)
    R = closed_forms.kron_gram(space, q, J.tolist())
    assert G.shape == R.shape == (shapes.dimension(space, q),) * 2
    assert np.abs(G - R).max() <= 1e-12 * np.abs(R).max()


def test_unit_cube_exact():
    """Exact rational Gram of the unit cube against the floating-point oracle."""
    q = (2, 1, 3)
    I3 = [[Fraction(int(i == j)) for j in range(3)] for i in range(3)]
    for space in SPACES:
        R = closed_forms.kron_gram(space, q, I3).astype(np.float64)
        G = og.gram(space, q, "affine", np.concatenate([np.zeros(3), np.eye(3).ravel()]))
        assert np.abs(G - R).max() <= 1e-13 * np.abs(R).max(), space


@pytest.mark.parametrize("space", SPACES)
def test_per_direction_rules_are_enough_on_affine_maps(space):
    q = (3, 1, 2)
    A = meshgen.affine_parallelepipeds(1, seed=510)[0]
    G = og.gram(space, q, "affine", A)                       # default: one rule per direction
    H = og.gram(space, q, "affine", A, L=max(q) + 2)         # one larger rule everywhere
    assert quadrature.default_points(space, q) == tuple(x if space == "L2" else x + 1 for x in q)
    assert np.abs(G - H).max() <= 1e-12 * np.abs(H).max()


@pytest.mark.parametrize("space", SPACES)
def test_uniform_triple_is_the_uniform_order(space):
    X = meshgen.perturbed_hexes(1, seed=520)[0]
    assert np.array_equal(og.gram(space, (2, 2, 2), "trilinear", X), og.gram(space, 2, "trilinear", X))


def test_cyclic_relabelling_permutes_the_gram():
    """Relabelling the master coordinates cyclically (xi1, xi2, xi3) ->
    (xi2, xi3, xi1), in the map and in the orders, keeps the orientation and
    renumbers the H1 basis: the Gram is the same matrix, rows and columns
    permuted."""
    q = (1, 3, 2)
    qs = (q[1], q[2], q[0])
    X = meshgen.perturbed_hexes(1, seed=530)[0]
    # new corner (v1, v2, v3) is old corner (v3, v1, v2); vertex index v1 + 2 v2 + 4 v3
    perm = [((v >> 2) & 1) | ((v & 1) << 1) | (((v >> 1) & 1) << 2) for v in range(8)]
    Xs = X[perm]
    G = og.gram("H1", q, "trilinear", X)
    Gs = og.gram("H1", qs, "trilinear", Xs)
    R1, R2, R3 = q[0] + 1, q[1] + 1, q[2] + 1
    # basis (i1, i2, i3) of q is basis (i2, i3, i1) of qs
    idx = [i2 + R2 * i3 + R2 * R3 * i1 for i3 in range(R3) for i2 in range(R2) for i1 in range(R1)]
    assert np.abs(Gs[np.ix_(idx, idx)] - G).max() <= 1e-12 * np.abs(G).max()
