"""Pins of the condensation oracle (Cholesky of packed Grams and solves with
the factor; Section 1 and (3.7)-(3.8)), CPU only.  Each pin comes from outside
the oracle's own column recurrence: a closed form, the uniqueness of the
factor, a library factorization, the Kronecker rule, or a constructed failure."""
import numpy as np
import pytest

import meshgen
from oracle import condense
from oracle import gram as og

EPS = np.finfo(np.float64).eps


def rand_upper(n, rng, lo=0.5, hi=2.0):
    U = np.triu(rng.standard_normal((n, n)), 1)
    U[np.diag_indices(n)] = rng.uniform(lo, hi, n)
    return U


def test_two_by_two_closed_form():
    a, b, c = 4.0, 2.0, 5.0
    U, info = condense.cholesky_upper(np.array([[a, b], [b, c]]))
    assert info == 0
    ref = np.array([[np.sqrt(a), b / np.sqrt(a)], [0.0, np.sqrt(c - b * b / a)]])
    assert np.allclose(U, ref, rtol=0, atol=4 * EPS)


@pytest.mark.parametrize("n", [1, 3, 17, 40])
def test_recovers_a_known_factor(n):
    """U with a positive diagonal is the unique factor of U^T U."""
    rng = np.random.default_rng(n)
    U0 = rand_upper(n, rng)
    up, info = condense.cholesky_packed(og.packed_upper(U0.T @ U0), n)
    assert info == 0
    U = condense.upper_from_packed(up, n)
    kappa = np.linalg.cond(U0.T @ U0)
    assert np.abs(U - U0).max() <= 8 * n * EPS * kappa * np.abs(U0).max()
    assert np.all(np.tril(U, -1) == 0)


def test_matches_library_factor():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((30, 30))
    G = M @ M.T + 30 * np.eye(30)
    U, info = condense.cholesky_upper(G)
    assert info == 0
    assert np.allclose(U, np.linalg.cholesky(G).T, rtol=0, atol=1e-13 * np.abs(U).max())


def test_kronecker_rule():
    """chol(A (x) B) = chol(A) (x) chol(B): the factor of a tensor-product Gram
    (the flat index of the spaces runs i1 fastest) is the product of 1D factors."""
    rng = np.random.default_rng(5)
    Ua, Ub, Uc = rand_upper(3, rng), rand_upper(4, rng), rand_upper(2, rng)
    A, B, C = Ua.T @ Ua, Ub.T @ Ub, Uc.T @ Uc
    U, info = condense.cholesky_upper(np.kron(C, np.kron(B, A)))
    assert info == 0
    ref = np.kron(Uc, np.kron(Ub, Ua))
    assert np.abs(U - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 2, 7, 20])
def test_info_names_the_first_failing_minor(k):
    """Make the pivot of column k - 1 exactly -1: leading minors of order < k
    stay positive definite, order k does not."""
    n = 20
    rng = np.random.default_rng(10 + k)
    U0 = rand_upper(n, rng)
    G = U0.T @ U0
    j = k - 1
    G[j, j] = U0[:j, j] @ U0[:j, j] - 1.0
    U, info = condense.cholesky_upper(G)
    assert info == k
    assert np.allclose(U[:, :j], U0[:, :j], rtol=0, atol=1e-10 * np.abs(U0).max())
    assert np.all(U[:, j:] == 0)


def test_info_special_cases():
    assert condense.cholesky_upper(np.zeros((4, 4)))[1] == 1
    assert condense.cholesky_upper(np.diag([1.0, 2.0, -1.0, 3.0]))[1] == 3
    assert condense.cholesky_upper(np.diag([1.0, np.nan, 1.0]))[1] == 2
    v = np.arange(1.0, 5.0)
    assert condense.cholesky_upper(np.outer(v, v))[1] == 2      # rank one: the second pivot is 0 (or rounds below)
    assert condense.cholesky_upper(np.array([[9.0]]))[0][0, 0] == 3.0


@pytest.mark.parametrize("m", [1, 5])
def test_solve_recovers_a_known_solution(m):
    n = 25
    rng = np.random.default_rng(20 + m)
    U0 = rand_upper(n, rng)
    G = U0.T @ U0
    X0 = rng.standard_normal((n, m))
    up, info = condense.cholesky_packed(og.packed_upper(G), n)
    X = condense.solve_packed(up, n, G @ X0)
    assert info == 0
    assert np.abs(X - X0).max() <= 16 * n * EPS * np.linalg.cond(G) * np.abs(X0).max()
    assert np.allclose(condense.solve_packed(up, n, G[:, 0]), np.eye(n)[:, 0], atol=1e-10)


@pytest.mark.parametrize("space,p", [("H1", 2), ("HCURL", 2), ("HDIV", 1), ("L2", 3)])
def test_element_grams_are_positive_definite(space, p):
    """The Grams of the four test inner products factor, and U^T U gives them back."""
    X = meshgen.perturbed_hexes(1, seed=300)[0]
    G = og.gram(space, p, "trilinear", X)
    n = G.shape[0]
    up, info = condense.cholesky_packed(og.packed_upper(G), n)
    assert info == 0
    U = condense.upper_from_packed(up, n)
    assert np.abs(U.T @ U - G).max() <= 8 * n * EPS * np.abs(G).max()
