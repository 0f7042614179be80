"""GPU parity of the condensation kernels (Cholesky factor of packed Grams and
solves with it; Section 1 and (3.7)-(3.8)) against the FP64 oracle, through
the C ABI.

Tolerances come from the perturbation theory of the factorization, since the
two sides sum in different orders.  Cholesky is backward stable, so
|U^T U - G| <= c n eps |G| whatever the conditioning (checked with c = 4), and
the factor itself moves by at most about kappa(G) times that, so U is compared
entry by entry within 4 n eps kappa(G) max|U|; the solution of G x = b within
8 n eps kappa(G) max|x|.  The failure index info is an integer and must match
exactly; the failing cases put a pivot at -1, far from any rounding.
"""
import numpy as np
import pytest
import torch

import meshgen
from oracle import condense
from oracle import gram as og

pytestmark = pytest.mark.gpu

EPS = {"fp64": np.finfo(np.float64).eps, "fp32": np.finfo(np.float32).eps}
DT = {"fp64": torch.float64, "fp32": torch.float32}


def say(*a):
    print("[gpu-condense]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def spd(n, rng):
    """Well conditioned SPD matrix (kappa of a few units)."""
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n)


def factor(ctx, Gs, prec="fp64"):
    """Packed Grams [E, n, n] -> (GPU packed factors [E, m] as float64, info [E])."""
    n = Gs.shape[1]
    ap = np.concatenate([og.packed_upper(G) for G in Gs])
    t = torch.from_numpy(ap).to(DT[prec]).cuda()
    info = torch.full((len(Gs),), -99, dtype=torch.int32, device="cuda")
    ctx.cholesky(t, n, info=info)
    torch.cuda.synchronize()
    return t.cpu().double().numpy().reshape(len(Gs), -1), info.cpu().numpy()


def check_factor(Up, G, prec, label):
    n = G.shape[0]
    U = condense.upper_from_packed(Up, n)
    R, info = condense.cholesky_upper(G)
    assert info == 0, label
    eps = EPS[prec]
    back = np.abs(U.T @ U - G).max() / np.abs(G).max()
    assert back <= 4 * n * eps, f"{label}: backward error {back:.3e}"
    kappa = np.linalg.cond(G)
    fwd = np.abs(U - R).max() / np.abs(R).max()
    assert fwd <= 4 * n * eps * kappa, f"{label}: |U - U_oracle| {fwd:.3e}, kappa {kappa:.2e}"
    assert np.all(np.tril(U, -1) == 0)


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 33, 64, 100, 129, 200, 257, 1000])
def test_factor_synthetic(ctx, n):
    say("factor synthetic", n)
    rng = np.random.default_rng(400 + n)
    E = 3
    Gs = np.stack([spd(n, rng) for _ in range(E)])
    for prec in ("fp64", "fp32"):
        G_in = Gs.astype(np.float32).astype(np.float64) if prec == "fp32" else Gs
        U, info = factor(ctx, G_in, prec)
        assert list(info) == [0] * E
        for e in range(E):
            check_factor(U[e], G_in[e], prec, f"n={n} {prec} e={e}")


@pytest.mark.parametrize("space,p", [("H1", 3), ("HCURL", 2), ("HDIV", 3), ("L2", 4), ("H1", 7)])
def test_factor_element_grams(ctx, dpg, space, p):
    """The Grams the integration kernels wrote, factored where they are."""
    say("factor grams", space, p)
    n = dpg.gram_dim(space, p)
    E = 3
    X = meshgen.perturbed_hexes(E, seed=410 + p)
    G = ctx.gram(space, p, torch.from_numpy(X).cuda())
    Gn = G.cpu().numpy().reshape(E, -1)
    info = torch.full((E,), -99, dtype=torch.int32, device="cuda")
    ctx.cholesky(G, n, info=info)
    torch.cuda.synchronize()
    U = G.cpu().numpy().reshape(E, -1)
    assert list(info.cpu().numpy()) == [0] * E
    for e in range(E):
        check_factor(U[e], og.unpack_upper(Gn[e], n), "fp64", f"{space} p={p} e={e}")


@pytest.mark.parametrize("n,k", [(48, 1), (48, 16), (48, 17), (48, 40), (130, 64), (130, 65), (130, 100)])
def test_failure_index(ctx, n, k):
    """A pivot of exactly -1 at column k-1; the other elements are untouched by it."""
    say("info", n, k)
    rng = np.random.default_rng(420 + k)
    Gs = np.stack([spd(n, rng) for _ in range(3)])
    R, _ = condense.cholesky_upper(Gs[1])
    j = k - 1
    Gs[1][j, j] = R[:j, j] @ R[:j, j] - 1.0
    assert condense.cholesky_upper(Gs[1])[1] == k
    for prec in ("fp64", "fp32"):
        G_in = Gs.astype(np.float32).astype(np.float64) if prec == "fp32" else Gs
        U, info = factor(ctx, G_in, prec)
        assert list(info) == [0, k, 0], prec
        for e in (0, 2):
            check_factor(U[e], G_in[e], prec, f"k={k} {prec} e={e}")
        if j:                                    # the finished columns before the failure
            Uf = condense.upper_from_packed(U[1], n)
            Rf, _ = condense.cholesky_upper(G_in[1])
            tol = 4 * n * EPS[prec] * np.linalg.cond(G_in[1][:j, :j])
            assert np.abs(Uf[:, :j] - Rf[:, :j]).max() <= tol * max(1.0, np.abs(Rf).max()), prec


def test_failure_special_cases(ctx):
    n = 20
    rng = np.random.default_rng(430)
    Gs = np.stack([spd(n, rng) for _ in range(3)])
    Gs[0][5, 5] = np.nan
    Gs[2] = 0.0
    _, info = factor(ctx, Gs)
    assert list(info) == [condense.cholesky_upper(G)[1] for G in Gs] == [6, 0, 1]


@pytest.mark.parametrize("n,nrhs", [(1, 1), (17, 1), (17, 16), (33, 21), (64, 40), (130, 7), (130, 70), (300, 19),
                                    (1000, 129)])
def test_solve(ctx, n, nrhs):
    say("solve", n, nrhs)
    rng = np.random.default_rng(440 + n + nrhs)
    E = 3
    Gs = np.stack([spd(n, rng) for _ in range(E)])
    for prec in ("fp64", "fp32"):
        G_in = Gs.astype(np.float32).astype(np.float64) if prec == "fp32" else Gs
        up = np.concatenate([condense.cholesky_packed(og.packed_upper(G), n)[0] for G in G_in])
        B = rng.standard_normal((E, nrhs, n))            # column-major n x nrhs per element
        if prec == "fp32":
            up = up.astype(np.float32).astype(np.float64)
            B = B.astype(np.float32).astype(np.float64)
        tu = torch.from_numpy(up).to(DT[prec]).cuda()
        tb = torch.from_numpy(B).to(DT[prec]).cuda()
        ctx.cholesky_solve(tu, n, tb)
        torch.cuda.synchronize()
        X = tb.cpu().double().numpy()
        m = n * (n + 1) // 2
        for e in range(E):
            R = condense.solve_packed(up[e * m:(e + 1) * m], n, B[e].T)
            kappa = np.linalg.cond(G_in[e])
            err = np.abs(X[e].T - R).max() / np.abs(R).max()
            assert err <= 8 * n * EPS[prec] * kappa, f"n={n} nrhs={nrhs} {prec} e={e}: {err:.3e}"


def test_factor_without_info_matches(ctx):
    """info is optional: the factor written without it is bit for bit the one written with it."""
    n = 200
    rng = np.random.default_rng(460)
    Gs = np.stack([spd(n, rng) for _ in range(2)])
    ap = np.concatenate([og.packed_upper(G) for G in Gs])
    for prec in ("fp64", "fp32"):
        t1 = torch.from_numpy(ap).to(DT[prec]).cuda()
        t2 = t1.clone()
        info = torch.full((2,), -99, dtype=torch.int32, device="cuda")
        ctx.cholesky(t1, n, info=info)
        ctx.cholesky(t2, n)
        torch.cuda.synchronize()
        assert list(info.cpu().numpy()) == [0, 0]
        assert torch.equal(t1, t2), prec


def test_solve_many_rhs_blocks(ctx):
    """Right-hand sides over several 64-column workgroups, the last one partial, against the
    oracle's solve and against solving the columns one block at a time."""
    n, nrhs = 200, 150
    rng = np.random.default_rng(470)
    G = spd(n, rng)
    up = condense.cholesky_packed(og.packed_upper(G), n)[0]
    B = rng.standard_normal((1, nrhs, n))
    tu = torch.from_numpy(up).cuda()
    tb = torch.from_numpy(B).cuda()
    ctx.cholesky_solve(tu, n, tb)
    parts = [torch.from_numpy(np.ascontiguousarray(B[:, c:c + 37])).cuda() for c in range(0, nrhs, 37)]
    for t in parts:
        ctx.cholesky_solve(tu, n, t)
    torch.cuda.synchronize()
    X = tb.cpu().numpy()[0]
    R = condense.solve_packed(up, n, B[0].T)
    err = np.abs(X.T - R).max() / np.abs(R).max()
    assert err <= 8 * n * EPS["fp64"] * np.linalg.cond(G), err
    # each column's result does not depend on which workgroup solved it
    Y = np.concatenate([t.cpu().numpy()[0] for t in parts], axis=0)
    assert np.abs(Y - X).max() <= 8 * n * EPS["fp64"] * np.linalg.cond(G) * np.abs(X).max()


def test_condensation_round_trip(ctx, dpg):
    """Factor H(div) p=3 Grams where they were integrated, solve G X = B with
    them, and check G X = B with the Grams recomputed."""
    space, p, E, nrhs = "HDIV", 3, 4, 27
    n = dpg.gram_dim(space, p)
    X = torch.from_numpy(meshgen.perturbed_hexes(E, seed=450)).cuda()
    G = ctx.gram(space, p, X)
    Gn = G.cpu().numpy().reshape(E, -1)
    ctx.cholesky(G, n)
    B = torch.randn(E, nrhs, n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    Bn = B.cpu().numpy()
    ctx.cholesky_solve(G, n, B)
    torch.cuda.synchronize()
    Xs = B.cpu().numpy()
    for e in range(E):
        Ge = og.unpack_upper(Gn[e], n)
        res = np.abs(Ge @ Xs[e].T - Bn[e].T).max() / np.abs(Bn[e]).max()
        assert res <= 8 * n * EPS["fp64"] * np.linalg.cond(Ge), (e, res)


def test_errors_and_empty(ctx, dpg):
    n = 8
    m = n * (n + 1) // 2
    ap = torch.zeros(2 * m, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.cholesky(ap[:m + 1], n)
    with pytest.raises(dpg.DpgError):                          # right-hand side overlaps the factor
        ctx.cholesky_solve(ap, n, ap[:2 * n])
    assert ctx.cholesky(torch.zeros(0, dtype=torch.float64, device="cuda"), n).numel() == 0
    rc = dpg._lib.dpg_cholesky_packed(ctx.handle, 1, 0, ap.data_ptr(), None, 0, None)
    assert rc == dpg.EINVAL
    rc = dpg._lib.dpg_cholesky_solve_packed(ctx.handle, 1, n, ap.data_ptr(), 0, ap.data_ptr(), 0, None)
    assert rc == dpg.EINVAL
    rc = dpg._lib.dpg_cholesky_packed(ctx.handle, 1, n, ap.data_ptr(), None, 7, None)
    assert rc == dpg.EINVAL
    # one element's packed matrix must stay addressable with 32-bit byte offsets
    rc = dpg._lib.dpg_cholesky_packed(ctx.handle, 1, 16385, ap.data_ptr(), None, 0, None)
    assert rc == dpg.EINVAL
    rc = dpg._lib.dpg_cholesky_solve_packed(ctx.handle, 1, 16385, ap.data_ptr(), 1, ap.data_ptr(), 0, None)
    assert rc == dpg.EINVAL


def test_benchmark_size_sampled(ctx, dpg):
    """The launch the benchmark times: 1024 H1 p = 7 Grams (n = 512) factored in
    place, then G^-1 B with 343 right-hand sides; sampled elements against the
    oracle."""
    space, p, E, nrhs = "H1", 7, 1024, 343
    n = dpg.gram_dim(space, p)
    X = meshgen.perturbed_hexes(E, noise=0.15, seed=1713)
    G = ctx.gram(space, p, torch.from_numpy(X).cuda())
    m = n * (n + 1) // 2
    picks = [0, 517, E - 1]
    Gs = {e: G[e * m:(e + 1) * m].cpu().numpy() for e in picks}
    info = torch.full((E,), -99, dtype=torch.int32, device="cuda")
    ctx.cholesky(G, n, info=info)
    B = torch.randn(E, nrhs, n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(11))
    Bs = {e: B[e].cpu().numpy() for e in picks}
    ctx.cholesky_solve(G, n, B)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    for e in picks:
        Ge = og.unpack_upper(Gs[e], n)
        check_factor(G[e * m:(e + 1) * m].cpu().numpy(), Ge, "fp64", f"benchmark e={e}")
        R = condense.solve_packed(condense.cholesky_packed(Gs[e], n)[0], n, Bs[e].T)
        err = np.abs(B[e].cpu().numpy().T - R).max() / np.abs(R).max()
        assert err <= 8 * n * EPS["fp64"] * np.linalg.cond(Ge), (e, err)
