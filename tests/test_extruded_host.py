"""Host checks of the extruded-element inputs (no GPU): the recipe draws maps of
the second form of (2.89), and their trilinear vertices describe the same map."""
import numpy as np

import meshgen


def trilinear_map(X, xi):
    """x(xi) = sum_v X_v prod_d (v_d ? xi_d : 1 - xi_d) for one element X [8, 3]."""
    c = meshgen.unit_corners()
    w = np.prod(np.where(c[None] > 0, xi[:, None, :], 1.0 - xi[:, None, :]), axis=2)
    return w @ X


def test_extruded_vertices_describe_an_extrusion():
    E = meshgen.extruded_prisms(7, seed=3)
    X = meshgen.extruded_as_trilinear(E)
    rng = np.random.default_rng(0)
    for e in range(7):
        xi = rng.uniform(size=(50, 3))
        x = trilinear_map(X[e], xi)
        # x1 = x1_0 + lambda1 xi1, independent of (xi2, xi3)
        assert np.allclose(x[:, 0], E[e, 0] + E[e, 1] * xi[:, 0], atol=1e-14)
        # (x2, x3) bilinear in (xi2, xi3) through the four cross-section corners, independent of xi1
        q = E[e, 2:].reshape(4, 2)
        a2, a3 = xi[:, 1:2], xi[:, 2:3]
        ref = (1 - a2) * (1 - a3) * q[0] + a2 * (1 - a3) * q[1] + (1 - a2) * a3 * q[2] + a2 * a3 * q[3]
        assert np.allclose(x[:, 1:], ref, atol=1e-14)


def test_extruded_recipe_ranges():
    E = meshgen.extruded_prisms(1000, noise=0.15, lam_lo=0.5, lam_hi=2.0, seed=4)
    assert E.shape == (1000, 10)
    assert E[:, 1].min() >= 0.5 and E[:, 1].max() <= 2.0
    q = E[:, 2:].reshape(-1, 4, 2)
    sq = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])
    assert np.abs(q - sq).max() <= 0.15
    assert np.array_equal(meshgen.extruded_prisms(3, seed=9), meshgen.extruded_prisms(3, seed=9))
