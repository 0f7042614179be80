"""GPU parity of the Grams of non-uniform orders (p1, p2, p3) (the text after
Algorithm 2: one Gauss rule per coordinate, least-order coordinate
outermost) against the FP64 oracle, through the C ABI.

Tolerances as for the uniform kernels: FP64 1e-12 (relative Frobenius and
max), FP32 2e-6 (relative Frobenius); both sides use the same per-direction
rules, so they differ by rounding only.
"""
import numpy as np
import pytest
import torch

import meshgen
from oracle import gram as og
from oracle import shapes

pytestmark = pytest.mark.gpu

SPACES = ["H1", "HCURL", "HDIV", "L2"]
TOL64 = 1e-12
FP32_REL = 2e-6


def say(*a):
    print("[gpu-aniso]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def run(ctx, space, q, geom, kind="trilinear", prec="fp64", nq=0, status=None, path="auto"):
    g = torch.from_numpy(np.ascontiguousarray(geom)).cuda()
    out = ctx.gram_aniso(space, q, g, kind=kind, prec=prec, nq=nq, status=status, path=path)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def elem(o, e, space, q):
    n = shapes.dimension(space, q)
    m = n * (n + 1) // 2
    return og.unpack_upper(o[e * m:(e + 1) * m].astype(np.float64), n)


def rel(G, R):
    return np.linalg.norm(G - R) / np.linalg.norm(R), np.abs(G - R).max() / np.abs(R).max()


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("q", [(1, 2, 3), (3, 1, 2), (2, 4, 1), (1, 1, 1), (3, 3, 2)])
def test_aniso_vs_oracle(ctx, space, q):
    """Both routes (the entry point's own, and the per-direction kernel forced) in FP64
    and FP32 against the oracle."""
    say(space, q, ctx.aniso_route(space, q))
    E = 3
    X = meshgen.perturbed_hexes(E, seed=600 + sum(q))
    for path in ("auto", "general"):
        o64 = run(ctx, space, q, X, path=path)
        o32 = run(ctx, space, q, X, prec="fp32", path=path)
        for e in range(E):
            R = og.gram(space, q, "trilinear", X[e])
            fro, mx = rel(elem(o64, e, space, q), R)
            assert fro <= TOL64 and mx <= TOL64, f"{space} {q} {path} e={e}: fro {fro:.3e} max {mx:.3e}"
            fro32, _ = rel(elem(o32, e, space, q), R)
            assert fro32 <= FP32_REL, f"{space} {q} {path} e={e} fp32: {fro32:.3e}"


@pytest.mark.parametrize("space,q", [("H1", (8, 5, 7)), ("HCURL", (6, 4, 5)), ("HDIV", (4, 6, 5)), ("L2", (8, 7, 6)),
                                     ("H1", (10, 9, 10)), ("HCURL", (9, 10, 8)), ("HDIV", (10, 8, 9)), ("L2", (10, 10, 9))])
def test_aniso_high_orders(ctx, space, q):
    """Full matrices up to 1000 unknowns; above that (the oracle's full Gram takes
    minutes there) the diagonal and 3000 random entries, computed one by one."""
    say("high", space, q)
    X = meshgen.perturbed_hexes(2, seed=610)
    o = run(ctx, space, q, X)
    n = shapes.dimension(space, q)
    rng = np.random.default_rng(611)
    for e in range(2):
        G = elem(o, e, space, q)
        if n <= 1000:
            R = og.gram(space, q, "trilinear", X[e])
            fro, mx = rel(G, R)
            assert fro <= TOL64 and mx <= TOL64, f"{space} {q} e={e}: fro {fro:.3e} max {mx:.3e}"
            continue
        I = np.concatenate([np.arange(n), rng.integers(0, n, 3000)])
        J = np.concatenate([np.arange(n), rng.integers(0, n, 3000)])
        R = og.gram_entries(space, q, "trilinear", X[e], I, J)
        err = np.abs(G[I, J] - R).max() / np.abs(G).max()
        assert err <= TOL64, f"{space} {q} e={e}: sampled max {err:.3e}"


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [2, 5])
def test_uniform_orders_match_the_uniform_kernels(ctx, space, p):
    """Equal orders: the per-direction kernel (path GENERAL) and the embedded route
    (an explicit nq equal to the default rule) against the uniform kernels, which the
    entry point itself takes for nq = 0 (bit for bit the uniform call)."""
    X = meshgen.perturbed_hexes(4, seed=620 + p)
    L = p if space == "L2" else p + 1
    assert ctx.aniso_route(space, (p, p, p)) == "uniform"
    assert ctx.aniso_route(space, (p, p, p), nq=L) == "embedded"
    a = run(ctx, space, (p, p, p), X, nq=L, path="general")
    b = run(ctx, space, (p, p, p), X, nq=L)
    d = run(ctx, space, (p, p, p), X)
    u = ctx.gram(space, p, torch.from_numpy(X).cuda(), path="general").cpu().numpy()
    assert np.array_equal(d, u)
    for e in range(4):
        for o in (a, b):
            fro, mx = rel(elem(o, e, space, (p,) * 3), elem(u, e, space, (p,) * 3))
            assert fro <= TOL64 and mx <= TOL64, f"{space} p={p} e={e}"


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("q,nq", [((4, 4, 3), 5), ((3, 3, 3), 2), ((5, 5, 5), 8), ((2, 2, 5), 8)])
def test_explicit_rule_routes(ctx, dpg, space, q, nq):
    """An explicit rule of nq points in every direction: embedded in the uniform
    kernel of an order whose default rule has at least nq points (padded with
    zero-weight points) where that carries at most about 16 times the entries,
    else the per-direction kernel; both against the oracle with the same rule, and
    dpg_gram_integrate with nq at equal orders against the aniso call."""
    want = "per-direction" if q == (2, 2, 5) else "embedded"
    assert ctx.aniso_route(space, q, nq=nq) == want
    X = meshgen.perturbed_hexes(2, seed=680 + nq)
    o = run(ctx, space, q, X, nq=nq)
    g = run(ctx, space, q, X, nq=nq, path="general")
    for e in range(2):
        R = og.gram(space, q, "trilinear", X[e], L=nq)
        for out in (o, g):
            fro, mx = rel(elem(out, e, space, q), R)
            assert fro <= TOL64 and mx <= TOL64, f"{space} {q} nq={nq} e={e}: {fro:.3e} {mx:.3e}"
    if len(set(q)) == 1:
        u = ctx.gram(space, q[0], torch.from_numpy(X).cuda(), nq=nq, path="general").cpu().numpy()
        assert np.array_equal(u, o)


# (8, 4, 4) and (6, 3, 3) skip whole x-tiles (j2 past the embedded range), (4, 8, 4) and
# L2 (3, 8, 4) whole y chunks (j1 past it)
EMBEDDED = [("H1", (7, 6, 5)), ("H1", (3, 1, 2)), ("H1", (10, 9, 8)), ("HCURL", (6, 5, 4)), ("HCURL", (2, 3, 1)),
            ("HDIV", (5, 6, 4)), ("HDIV", (4, 4, 2)), ("L2", (8, 7, 6)), ("L2", (3, 2, 1)), ("H1", (8, 4, 4)),
            ("HDIV", (6, 3, 3)), ("H1", (4, 8, 4)), ("L2", (3, 8, 4))]


@pytest.mark.parametrize("space,q", EMBEDDED)
def test_embedded_route(ctx, space, q):
    """Orders embedded in the uniform kernel of order max p_d (each direction on its
    own rule, padded with zero-weight points; only the submatrix's entries stored)
    against the oracle and against the per-direction kernel, FP64 and FP32."""
    say("embedded", space, q)
    assert ctx.aniso_route(space, q) == "embedded"
    assert ctx.aniso_route(space, q, path="general") == "per-direction"
    n = shapes.dimension(space, q)
    E = 3 if n <= 400 else 2
    X = meshgen.perturbed_hexes(E, seed=700 + sum(q))
    a = run(ctx, space, q, X)
    g = run(ctx, space, q, X, path="general")
    a32 = run(ctx, space, q, X, prec="fp32")
    for e in range(E):
        R = og.gram(space, q, "trilinear", X[e])
        fro, mx = rel(elem(a, e, space, q), R)
        assert fro <= TOL64 and mx <= TOL64, f"{space} {q} e={e}: fro {fro:.3e} max {mx:.3e}"
        fro, mx = rel(elem(a, e, space, q), elem(g, e, space, q))
        assert fro <= TOL64 and mx <= TOL64, f"{space} {q} e={e} vs per-direction: {fro:.3e} {mx:.3e}"
        fro32, _ = rel(elem(a32, e, space, q), R)
        assert fro32 <= FP32_REL, f"{space} {q} e={e} fp32: {fro32:.3e}"


def test_embedded_geometry_kinds(ctx):
    """The embedded route on affine and extruded maps (the uniform kernel's metric
    for each kind, with the per-direction points)."""
    q = (4, 3, 2)
    for space in SPACES:
        assert ctx.aniso_route(space, q) == "embedded", space
        A = meshgen.affine_parallelepipeds(2, seed=710)
        o = run(ctx, space, q, A, kind="affine")
        for e in range(2):
            fro, mx = rel(elem(o, e, space, q), og.gram(space, q, "affine", A[e]))
            assert fro <= TOL64 and mx <= TOL64, (space, e)
        Ex = meshgen.extruded_prisms(2, seed=711)
        o = run(ctx, space, q, Ex, kind="extruded")
        T = meshgen.extruded_as_trilinear(Ex)
        for e in range(2):
            fro, mx = rel(elem(o, e, space, q), og.gram(space, q, "trilinear", T[e]))
            assert fro <= TOL64 and mx <= TOL64, (space, e)


def test_embedded_high_order_batch(ctx, dpg):
    """H(curl) (10, 9, 9), 90 elements (several slab groups per element, the largest
    order of the embedded kernels): every element against the per-direction kernel,
    and sampled entries of two elements against the oracle."""
    space, q, E = "HCURL", (10, 9, 9), 90
    assert ctx.aniso_route(space, q) == "embedded"
    X = meshgen.perturbed_hexes(E, seed=720)
    g = torch.from_numpy(X).cuda()
    a = ctx.gram_aniso(space, q, g)
    b = ctx.gram_aniso(space, q, g, path="general")
    torch.cuda.synchronize()
    n = dpg.gram_dim_aniso(space, q)
    m = n * (n + 1) // 2
    A, B = a.view(E, m), b.view(E, m)
    err = ((A - B).abs().amax(dim=1) / B.abs().amax(dim=1)).max().item()
    say("HCURL (10, 9, 9): max rel diff vs per-direction", err)
    assert err <= TOL64
    rng = np.random.default_rng(721)
    for e in (3, 85):
        G = og.unpack_upper(A[e].cpu().numpy(), n)
        I = np.concatenate([np.arange(n), rng.integers(0, n, 2000)])
        J = np.concatenate([np.arange(n), rng.integers(0, n, 2000)])
        R = og.gram_entries(space, q, "trilinear", X[e], I, J)
        assert np.abs(G[I, J] - R).max() / np.abs(G).max() <= TOL64, e


@pytest.mark.parametrize("space", SPACES)
def test_one_rule_for_all_directions(ctx, space):
    """nq > 0: the same nq-point rule in every direction (the shortcut of
    using the largest rule everywhere)."""
    q = (2, 4, 3)
    X = meshgen.perturbed_hexes(2, seed=630)
    o = run(ctx, space, q, X, nq=6)
    for e in range(2):
        R = og.gram(space, q, "trilinear", X[e], L=6)
        fro, mx = rel(elem(o, e, space, q), R)
        assert fro <= TOL64 and mx <= TOL64, f"{space} e={e}"


@pytest.mark.parametrize("space", SPACES)
def test_affine_and_extruded_geometry(ctx, space):
    q = (3, 2, 4)
    A = meshgen.affine_parallelepipeds(2, seed=640)
    o = run(ctx, space, q, A, kind="affine")
    for e in range(2):
        fro, mx = rel(elem(o, e, space, q), og.gram(space, q, "affine", A[e]))
        assert fro <= TOL64 and mx <= TOL64
    Ex = meshgen.extruded_prisms(2, seed=641)
    o = run(ctx, space, q, Ex, kind="extruded")
    T = meshgen.extruded_as_trilinear(Ex)
    for e in range(2):
        fro, mx = rel(elem(o, e, space, q), og.gram(space, q, "trilinear", T[e]))
        assert fro <= TOL64 and mx <= TOL64


def test_cyclic_relabelling(ctx):
    """Relabelling (xi1, xi2, xi3) -> (xi2, xi3, xi1) in the map and the orders
    permutes the H1 basis, which changes the contraction order chosen for the
    least-order direction; the GPU results must agree after renumbering."""
    q = (2, 5, 3)
    qs = (q[1], q[2], q[0])
    X = meshgen.perturbed_hexes(1, seed=650)[0]
    perm = [((v >> 2) & 1) | ((v & 1) << 1) | (((v >> 1) & 1) << 2) for v in range(8)]
    G = elem(run(ctx, "H1", q, X[None]), 0, "H1", q)
    Gs = elem(run(ctx, "H1", qs, X[perm][None]), 0, "H1", qs)
    R1, R2, R3 = q[0] + 1, q[1] + 1, q[2] + 1
    idx = [i2 + R2 * i3 + R2 * R3 * i1 for i3 in range(R3) for i2 in range(R2) for i1 in range(R1)]
    fro, mx = rel(Gs[np.ix_(idx, idx)], G)
    assert fro <= TOL64 and mx <= TOL64


def test_bad_element_empty_and_errors(ctx, dpg):
    """Both routes (embedded by default, per-direction forced) flag and zero a bad element."""
    q = (2, 3, 1)
    X = meshgen.perturbed_hexes(3, seed=660)
    X[1] = X[1][[1, 0, 2, 3, 4, 5, 6, 7]]                  # swap two vertices: det J < 0 somewhere
    st = torch.full((3,), 7, dtype=torch.int32, device="cuda")
    for space, path in (("H1", "auto"), ("HDIV", "auto"), ("H1", "general"), ("HDIV", "general")):
        st.fill_(7)
        o = run(ctx, space, q, X, status=st, path=path)
        assert list(st.cpu().numpy()) == [0, dpg.EJACOBIAN, 0], (space, path)
        m = dpg.gram_dim_aniso(space, q)
        m = m * (m + 1) // 2
        assert np.all(o[m:2 * m] == 0)
        fro, _ = rel(elem(o, 2, space, q), og.gram(space, q, "trilinear", X[2]))
        assert fro <= TOL64
    empty = torch.empty((0,), dtype=torch.float64, device="cuda")
    assert ctx.gram_aniso("H1", q, empty).numel() == 0
    g = torch.from_numpy(meshgen.perturbed_hexes(1, seed=661)).cuda()
    for bad in ((0, 1, 1), (1, 11, 1)):
        with pytest.raises(dpg.DpgError):
            ctx.gram_aniso("H1", bad, g)
        with pytest.raises(dpg.DpgError):
            ctx.aniso_route("H1", bad)
    with pytest.raises(dpg.DpgError):
        ctx.gram_aniso("H1", q, g, nq=12)


def test_benchmark_size_sampled(ctx, dpg):
    """The launch the benchmark times for non-uniform orders: 4096 hexes, H1
    (7, 6, 5); sampled elements against the oracle."""
    q, E = (7, 6, 5), 4096
    X = meshgen.perturbed_hexes(E, noise=0.15, seed=1712)
    o = ctx.gram_aniso("H1", q, torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    n = dpg.gram_dim_aniso("H1", q)
    m = n * (n + 1) // 2
    for e in (0, 2049, E - 1):
        G = og.unpack_upper(o[e * m:(e + 1) * m].cpu().numpy(), n)
        fro, mx = rel(G, og.gram("H1", q, "trilinear", X[e]))
        assert fro <= TOL64 and mx <= TOL64, (e, fro, mx)
