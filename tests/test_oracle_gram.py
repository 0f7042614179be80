"""Pins of the brute-force Gram oracle (3D layer).

Each check is fixed by something other than the oracle's own formulas:

* textbook trilinear (p = 1) mass and stiffness matrices on the unit cube;
* the exact H1 Gram of the cube (0,2)^3 at p = 3 (worked example of the
  benchmark's first configuration) from the closed-form chart, stored in
  tests/golden/h1_cube2_p3_exact.txt;
* L2 on a scaled cube: diagonal by Legendre orthogonality (2.95);
* affine elements: brute force (quadrature of Piola-mapped shape functions)
  equals the Kronecker form built from the paper's chart (two independent
  routes), in all four spaces;
* exact-sequence relations (2.1): grad W in Q, curl Q in V, div V in Y with
  combinatorial incidence matrices, on distorted trilinear elements, plus
  curl grad = 0 and div curl = 0;
* constants lie in W and have zero gradient; the volume equals a surface
  integral by the divergence theorem;
* symmetry and positive definiteness; invariance under raising L for
  affine maps; entry-wise, mat-vec and packed forms agree with the full matrix.
"""
from fractions import Fraction

import numpy as np
import pytest

import meshgen
from oracle import closed_forms, geometry, gram, quadrature, shapes

SPACES = ["H1", "HCURL", "HDIV", "L2"]
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                    "h1_cube2_p3_exact.txt")


def random_hex(seed, noise=0.15):
    return meshgen.perturbed_hexes(1, noise=noise, seed=seed)[0]


def random_affine(seed):
    return meshgen.affine_parallelepipeds(1, seed=seed)[0]


# --------------------------------------------------------------------------
# textbook and worked examples
# --------------------------------------------------------------------------

def test_h1_p1_unit_cube_textbook():
    # P1 Lagrange on (0,1): L_0 = 1 - x, L_1 = x.  Mass [[1/3,1/6],[1/6,1/3]],
    # stiffness [[1,-1],[-1,1]]; the trilinear Gram is the Kronecker sum.
    M = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    K = np.array([[1.0, -1.0], [-1.0, 1.0]])
    kr = lambda a, b, c: np.kron(c, np.kron(b, a))
    ref = kr(M, M, M) + kr(K, M, M) + kr(M, K, M) + kr(M, M, K)
    G = gram.gram("H1", 1, "trilinear", meshgen.unit_corners())
    np.testing.assert_allclose(G, ref, atol=1e-15)


def load_golden():
    n = 64
    G = np.zeros((n, n), dtype=object)
    G[:, :] = Fraction(0)
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            I, J, v = line.split()
            G[int(I), int(J)] = G[int(J), int(I)] = Fraction(v)
    return G


def test_config1_cube2_h1_p3_exact_values():
    G = gram.gram("H1", 3, "trilinear", meshgen.scaled_cube(2.0)[0])
    ex = load_golden()
    # values quoted for the worked example
    assert ex[0, 0] == Fraction(26, 27) and ex[1, 0] == Fraction(4, 27)
    assert ex[21, 21] == Fraction(26, 27) and ex[63, 63] == Fraction(13, 463050)
    assert sum(ex[i, i] for i in range(64)) == Fraction(11981488, 1157625)
    assert int((ex != 0).sum()) == 2744
    exf = ex.astype(np.float64)
    assert np.abs(G - exf).max() <= 2e-15 * np.abs(exf).max()
    # exact zeros stay (numerically) zero
    assert np.abs(G[ex == 0]).max() < 1e-15


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_l2_scaled_cube_orthogonality(p):
    G = gram.gram("L2", p, "trilinear", meshgen.scaled_cube(2.0)[0])
    idx = shapes.basis_index("L2", p)
    ref = np.diag([1.0 / 8.0 / np.prod([2 * i + 1 for i in row[1:]]) for row in idx])
    np.testing.assert_allclose(G, ref, atol=1e-15)


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_affine_bruteforce_equals_closed_form(space, p):
    A = random_affine(100 + p)
    J = A[3:].reshape(3, 3)
    G = gram.gram(space, p, "affine", A, w0=0.7, w1=1.3)
    K = closed_forms.kron_gram(space, p, J, w0=0.7, w1=1.3)
    assert np.abs(G - K).max() <= 1e-13 * np.abs(K).max()
    # the same element given by its 8 vertices
    X = meshgen.affine_as_trilinear(A[None])[0]
    G2 = gram.gram(space, p, "trilinear", X, w0=0.7, w1=1.3)
    assert np.abs(G2 - K).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("space", SPACES)
def test_affine_invariant_under_more_points(space):
    A = random_affine(7)
    L0 = quadrature.default_points(space, 3)
    G0 = gram.gram(space, 3, "affine", A, L=L0)
    G1 = gram.gram(space, 3, "affine", A, L=L0 + 2)
    assert np.abs(G0 - G1).max() <= 1e-13 * np.abs(G0).max()


def test_trilinear_depends_on_points():
    # rational integrands: a different rule gives a (slightly) different matrix
    X = random_hex(3)
    G0 = gram.gram("H1", 3, "trilinear", X, L=4)
    G1 = gram.gram("H1", 3, "trilinear", X, L=6)
    d = np.abs(G0 - G1).max() / np.abs(G0).max()
    assert 1e-10 < d < 1e-2


# --------------------------------------------------------------------------
# exact sequence
# --------------------------------------------------------------------------

def _d1(k):
    """chi'_k = sign * nu_m: (m, sign), from chi'_0 = -1 = -nu_0, chi'_k = nu_{k-1}."""
    return (0, -1.0) if k == 0 else (k - 1, 1.0)


def incidence_grad(p):
    nW, nQ = shapes.dimension("H1", p), shapes.dimension("HCURL", p)
    D = np.zeros((nQ, nW))
    for I, (_, i1, i2, i3) in enumerate(shapes.basis_index("H1", p)):
        ii = [i1, i2, i3]
        for c in range(3):
            m, sg = _d1(ii[c])
            k = list(ii)
            k[c] = m
            D[shapes.flat_index("HCURL", p, c, *k), I] += sg
    return D


def incidence_curl(p):
    nQ, nV = shapes.dimension("HCURL", p), shapes.dimension("HDIV", p)
    D = np.zeros((nV, nQ))
    for I, (a, k1, k2, k3) in enumerate(shapes.basis_index("HCURL", p)):
        k = [k1, k2, k3]
        a1, a2 = (a + 1) % 3, (a + 2) % 3
        # curl(f e_a) = d_{a+2} f e_{a+1} - d_{a+1} f e_{a+2}   (2.67)
        m, sg = _d1(k[a2])
        kk = list(k)
        kk[a2] = m
        D[shapes.flat_index("HDIV", p, a1, *kk), I] += sg
        m, sg = _d1(k[a1])
        kk = list(k)
        kk[a1] = m
        D[shapes.flat_index("HDIV", p, a2, *kk), I] -= sg
    return D


def incidence_div(p):
    nV, nY = shapes.dimension("HDIV", p), shapes.dimension("L2", p)
    D = np.zeros((nY, nV))
    for I, (a, i1, i2, i3) in enumerate(shapes.basis_index("HDIV", p)):
        ii = [i1, i2, i3]
        m, sg = _d1(ii[a])
        ii[a] = m
        D[shapes.flat_index("L2", p, 0, *ii), I] += sg
    return D


@pytest.mark.parametrize("p", [1, 2, 3])
def test_exact_sequence_relations(p):
    X = random_hex(10 + p)
    L = p + 1
    G = lambda sp, w0, w1: gram.gram(sp, p, "trilinear", X, L=L, w0=w0, w1=w1)
    Dg, Dc, Dd = incidence_grad(p), incidence_curl(p), incidence_div(p)
    rel = lambda A, B: np.abs(A - B).max() / max(np.abs(B).max(), 1e-300)
    h1_grad = G("H1", 0.0, 1.0)
    curl_mass, curl_curl = G("HCURL", 1.0, 0.0), G("HCURL", 0.0, 1.0)
    div_mass, div_div = G("HDIV", 1.0, 0.0), G("HDIV", 0.0, 1.0)
    l2 = G("L2", 1.0, 0.0)
    assert rel(Dg.T @ curl_mass @ Dg, h1_grad) < 1e-13
    assert rel(Dc.T @ div_mass @ Dc, curl_curl) < 1e-13
    assert rel(Dd.T @ l2 @ Dd, div_div) < 1e-13
    assert np.abs(curl_curl @ Dg).max() < 1e-13 * np.abs(curl_curl).max()
    assert np.abs(div_div @ Dc).max() < 1e-13 * np.abs(div_div).max()


def hex_volume_divergence_theorem(X):
    """V = (1/3) sum over the 6 bilinear faces of int x . n dA (3x3 Gauss per face)."""
    z, w = np.polynomial.legendre.leggauss(3)
    z, w = 0.5 * (z + 1), 0.5 * w
    U, Vv = np.meshgrid(z, z, indexing="ij")
    W = np.outer(w, w)
    vol = 0.0
    for d in range(3):
        e1, e2 = (d + 1) % 3, (d + 2) % 3
        for side, sgn in ((0.0, -1.0), (1.0, 1.0)):
            xi = np.zeros((U.size, 3))
            xi[:, d] = side
            xi[:, e1] = U.ravel()
            xi[:, e2] = Vv.ravel()
            x = geometry.trilinear_map(X, xi)
            # tangents by exact differences (the map is linear in each variable)
            xa = xi.copy(); xa[:, e1] = 0.0
            xb = xi.copy(); xb[:, e1] = 1.0
            tu = geometry.trilinear_map(X, xb) - geometry.trilinear_map(X, xa)
            xa = xi.copy(); xa[:, e2] = 0.0
            xb = xi.copy(); xb[:, e2] = 1.0
            tv = geometry.trilinear_map(X, xb) - geometry.trilinear_map(X, xa)
            n = np.cross(tu, tv)
            vol += sgn * np.sum(W.ravel() * np.einsum("qi,qi->q", x, n)) / 3.0
    return vol


@pytest.mark.parametrize("p", [1, 2, 4])
def test_constants_and_volume(p):
    X = random_hex(20 + p)
    idx = shapes.basis_index("H1", p)
    c = np.all(idx[:, 1:] <= 1, axis=1).astype(float)
    G_mass = gram.gram("H1", p, "trilinear", X, w0=1.0, w1=0.0)
    G_grad = gram.gram("H1", p, "trilinear", X, w0=0.0, w1=1.0)
    assert np.abs(G_grad @ c).max() < 1e-13 * np.abs(G_grad).max()
    vol = hex_volume_divergence_theorem(X)
    assert abs(c @ G_mass @ c - vol) < 1e-13 * vol


# --------------------------------------------------------------------------
# structure
# --------------------------------------------------------------------------

@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_symmetric_positive_definite(space, p):
    X = random_hex(30 + p)
    G = gram.gram(space, p, "trilinear", X)
    assert G.shape == (shapes.dimension(space, p),) * 2
    assert np.abs(G - G.T).max() <= 1e-14 * np.abs(G).max()
    np.linalg.cholesky(G)
    assert np.linalg.eigvalsh(G).min() > 0


def test_dimensions():
    for p in range(1, 12):
        assert shapes.dimension("H1", p) == (p + 1) ** 3
        assert shapes.dimension("L2", p) == p ** 3
        assert shapes.dimension("HCURL", p) == 3 * p * (p + 1) ** 2
        assert shapes.dimension("HDIV", p) == 3 * (p + 1) * p ** 2


@pytest.mark.parametrize("space", SPACES)
def test_entries_matvec_packed_agree(space):
    p = 3
    X = random_hex(40)
    G = gram.gram(space, p, "trilinear", X, w0=0.9, w1=1.1)
    n = G.shape[0]
    rng = np.random.default_rng(1)
    I = rng.integers(0, n, 50)
    J = rng.integers(0, n, 50)
    e = gram.gram_entries(space, p, "trilinear", X, I, J, w0=0.9, w1=1.1)
    np.testing.assert_allclose(e, G[I, J], rtol=1e-13, atol=1e-15 * np.abs(G).max())
    r = rng.standard_normal(n)
    mv = gram.gram_matvec(space, p, "trilinear", X, r, w0=0.9, w1=1.1)
    np.testing.assert_allclose(mv, G @ r, rtol=1e-12, atol=1e-13 * np.abs(G @ r).max())
    ap = gram.packed_upper(G)
    assert ap.size == n * (n + 1) // 2
    Ii, Jj = np.triu_indices(n)
    np.testing.assert_array_equal(ap[gram.packed_offset(Ii, Jj)], G[Ii, Jj])
    np.testing.assert_allclose(gram.unpack_upper(ap, n), (G + G.T) / 2, rtol=0, atol=1e-14 * np.abs(G).max())


def test_jacobian_flag():
    X = meshgen.unit_corners().copy()
    assert gram.jacobian_ok("H1", 2, "trilinear", X)
    Xf = X.copy()
    Xf[[0, 7]] = Xf[[7, 0]]          # fold the element through itself
    assert not gram.jacobian_ok("H1", 2, "trilinear", Xf)
    A = np.zeros(12)
    A[3:] = np.diag([1.0, -1.0, 1.0]).ravel()
    assert not gram.jacobian_ok("H1", 2, "affine", A)
