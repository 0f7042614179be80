"""GPU parity of the HIP path against the FP64 CPU oracle (through the C ABI).

Tolerances (written here, derived in the design doc):
* FP64: ||G_gpu - G_oracle||_F <= 1e-12 ||G_oracle||_F and
        max |G_gpu - G_oracle| <= 1e-12 max |G_oracle|.
* FP32: ||G_gpu - G_oracle||_F <= FP32_REL ||G_oracle||_F.
Element-wise relative error is not used: many entries are exact zeros.
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
FP32_REL = 5e-7     # twice the largest error measured against the oracle (FP32 error table)


def say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    say("building tables")
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def run(ctx, space, p, geom_np, kind="trilinear", prec="fp64", path="auto", w0=1.0, w1=1.0, status=None, nq=0):
    g = torch.from_numpy(np.ascontiguousarray(geom_np)).cuda()
    out = ctx.gram(space, p, g, kind=kind, prec=prec, path=path, w0=w0, w1=w1, status=status, nq=nq)
    torch.cuda.synchronize()
    return out


def elem(out_np, e, space, p):
    n = shapes.dimension(space, p)
    m = n * (n + 1) // 2
    return og.unpack_upper(out_np[e * m:(e + 1) * m].astype(np.float64), n)


def compare64(G, R, what):
    fro = np.linalg.norm(G - R) / np.linalg.norm(R)
    mx = np.abs(G - R).max() / np.abs(R).max()
    assert fro <= TOL64 and mx <= TOL64, f"{what}: rel fro {fro:.3e}, rel max {mx:.3e}"
    return fro


def sampled_pairs(n, seed, k=3000):
    """The whole diagonal plus k random upper-triangle entries (I <= J)."""
    rng = np.random.default_rng(seed)
    I = rng.integers(0, n, k)
    J = rng.integers(0, n, k)
    I, J = np.minimum(I, J), np.maximum(I, J)
    return np.concatenate([I, np.arange(n)]), np.concatenate([J, np.arange(n)])


def compare_sampled(out_np, e, space, p, kind, geom, seed, what, tol=TOL64, L=None):
    """Entries of element e's packed output against the oracle computed one by one
    (og.gram_entries), on the diagonal and 3000 random entries: relative error in
    the Frobenius norm of the sample and (FP64) in its largest entry."""
    n = shapes.dimension(space, p)
    m = n * (n + 1) // 2
    I, J = sampled_pairs(n, seed)
    ref = og.gram_entries(space, p, kind, geom, I, J, L=L)
    got = out_np[e * m:(e + 1) * m][og.packed_offset(I, J)].astype(np.float64)
    fro = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    mx = np.abs(got - ref).max() / np.abs(ref).max()
    if tol == TOL64:
        assert fro <= tol and mx <= tol, f"{what}: sampled rel fro {fro:.3e}, rel max {mx:.3e}"
    else:
        assert fro <= tol, f"{what}: sampled rel fro {fro:.3e}"
    return fro


# --------------------------------------------------------------------------

def test_config1_cube_exact(ctx):
    say("config 1: cube (0,2)^3, H1 p=3")
    from tests.test_oracle_gram import load_golden
    ex = load_golden().astype(np.float64)
    X = meshgen.scaled_cube(2.0)
    out = run(ctx, "H1", 3, X).cpu().numpy()
    G = elem(out, 0, "H1", 3)
    assert np.abs(G - ex).max() <= 4e-15 * np.abs(ex).max()
    assert np.abs(G[ex == 0]).max() <= 4e-15
    R = og.gram("H1", 3, "trilinear", X[0])
    compare64(G, R, "config1 vs oracle")
    # the same cube as an affine map, reduced path
    A = np.zeros((1, 12))
    A[0, 3:] = (2.0 * np.eye(3)).ravel()
    Gr = elem(run(ctx, "H1", 3, A, kind="affine").cpu().numpy(), 0, "H1", 3)
    assert np.abs(Gr - ex).max() <= 4e-15 * np.abs(ex).max()


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_general_fp64(ctx, space, p):
    say(f"general fp64 {space} p={p}")
    X = meshgen.perturbed_hexes(3, seed=500 + 10 * p + SPACES.index(space))
    out = run(ctx, space, p, X).cpu().numpy()
    for e in range(3):
        compare64(elem(out, e, space, p), og.gram(space, p, "trilinear", X[e]), f"{space} p={p} e={e}")


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [7, 8])
def test_general_fp64_p7_p8(ctx, space, p):
    """Orders 7 and 8 on perturbed trilinear hexes, every space: full matrices where
    n <= 1000 (H1, L2), the diagonal and 3000 entries computed one by one above."""
    say(f"general fp64 {space} p={p}")
    X = meshgen.perturbed_hexes(3, seed=700 + 10 * p + SPACES.index(space))
    out = run(ctx, space, p, X).cpu().numpy()
    n = shapes.dimension(space, p)
    for e in (0, 2):
        if n <= 1000:
            compare64(elem(out, e, space, p), og.gram(space, p, "trilinear", X[e]), f"{space} p={p} e={e}")
        else:
            compare_sampled(out, e, space, p, "trilinear", X[e], seed=e, what=f"{space} p={p} e={e}")
    assert np.isfinite(out).all()


@pytest.mark.parametrize("space", SPACES)
def test_general_weights(ctx, space):
    say(f"general fp64 weighted {space}")
    p = 3
    X = meshgen.perturbed_hexes(2, seed=77)
    for w0, w1 in ((0.7, 1.3), (1.0, 0.0), (0.0, 1.0)):
        out = run(ctx, space, p, X, w0=w0, w1=w1).cpu().numpy()
        for e in range(2):
            R = og.gram(space, p, "trilinear", X[e], w0=w0, w1=w1)
            if np.abs(R).max() == 0:
                assert np.abs(elem(out, e, space, p)).max() == 0
                continue
            compare64(elem(out, e, space, p), R, f"{space} w=({w0},{w1})")


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [2, 4, 7])
def test_general_fp32(ctx, space, p):
    say(f"general fp32 {space} p={p}")
    X = meshgen.perturbed_hexes(2, seed=900 + p)
    out = run(ctx, space, p, X, prec="fp32").cpu().numpy()
    assert out.dtype == np.float32
    for e in range(2):
        R = og.gram(space, p, "trilinear", X[e])
        G = elem(out, e, space, p)
        fro = np.linalg.norm(G - R) / np.linalg.norm(R)
        say(f"  fp32 {space} p={p} e={e} rel fro {fro:.3e}")
        assert fro <= FP32_REL


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [1, 2, 3, 5, 6])
def test_reduced_fp64(ctx, space, p):
    say(f"reduced fp64 {space} p={p}")
    A = meshgen.affine_parallelepipeds(3, seed=300 + p)
    out = run(ctx, space, p, A, kind="affine", path="reduced").cpu().numpy()
    outg = run(ctx, space, p, A, kind="affine", path="general").cpu().numpy()
    for e in range(3):
        R = og.gram(space, p, "affine", A[e])
        compare64(elem(out, e, space, p), R, f"reduced {space} p={p}")
        compare64(elem(outg, e, space, p), R, f"general-affine {space} p={p}")
        compare64(elem(out, e, space, p), elem(outg, e, space, p), "reduced vs general")


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [7, 8])
def test_reduced_fp64_p7_p8(ctx, space, p):
    """The reduced (constant-Jacobian) path and the quadrature path on the same
    sheared parallelepipeds at orders 7 and 8: each against sampled oracle
    entries, and against each other over every entry."""
    say(f"reduced fp64 {space} p={p}")
    A = meshgen.affine_parallelepipeds(3, seed=310 + p)
    red = run(ctx, space, p, A, kind="affine", path="reduced").cpu().numpy()
    gen = run(ctx, space, p, A, kind="affine", path="general").cpu().numpy()
    for e in (0, 2):
        compare_sampled(red, e, space, p, "affine", A[e], seed=10 + e, what=f"reduced {space} p={p} e={e}")
        compare_sampled(gen, e, space, p, "affine", A[e], seed=10 + e, what=f"general-affine {space} p={p} e={e}")
    d = np.abs(red - gen).max() / np.abs(red).max()
    assert d <= TOL64, f"reduced vs general {space} p={p}: {d:.3e}"


@pytest.mark.parametrize("space", SPACES)
def test_nq_rule_invariance_affine(ctx, dpg, space):
    """On affine elements the default rule is exact (text after (2.22)), so raising
    the point count through dpg_gram_integrate (nq) leaves every Gram unchanged up
    to rounding; AUTO with nq takes the quadrature path as well."""
    say(f"nq invariance {space}")
    for p in (3, 6):
        A = meshgen.affine_parallelepipeds(3, seed=40 + p)
        ref = run(ctx, space, p, A, kind="affine", path="general").cpu().numpy()
        L = dpg.default_points(space, p)
        for nq in (L + 1, L + 2):
            for path in ("general", "auto"):
                out = run(ctx, space, p, A, kind="affine", path=path, nq=nq).cpu().numpy()
                d = np.abs(out - ref).max() / np.abs(ref).max()
                say(f"  {space} p={p} nq={nq} {path}: max rel change {d:.2e}")
                assert d <= TOL64


@pytest.mark.parametrize("space", SPACES)
def test_nq_rule_trilinear_vs_oracle(ctx, dpg, space):
    """On trilinear maps the integrands are rational and G depends on the rule: a
    requested nq must give the oracle's sum with exactly that rule, below and
    above the default."""
    say(f"nq trilinear {space}")
    p = 3
    X = meshgen.perturbed_hexes(2, seed=61)
    L = dpg.default_points(space, p)
    for nq in (L - 1, L + 2):
        out = run(ctx, space, p, X, nq=nq).cpu().numpy()
        for e in range(2):
            compare64(elem(out, e, space, p), og.gram(space, p, "trilinear", X[e], L=nq), f"{space} nq={nq}")
        default = run(ctx, space, p, X).cpu().numpy()
        assert np.abs(out - default).max() > 0          # a different rule, a different sum


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [9, 10, 11])
def test_high_order_sampled(ctx, space, p):
    say(f"high order sampled {space} p={p}")
    X = meshgen.perturbed_hexes(1, seed=1100 + p)
    out = run(ctx, space, p, X).cpu().numpy()
    n = shapes.dimension(space, p)
    rng = np.random.default_rng(p)
    I = rng.integers(0, n, 3000)
    J = rng.integers(0, n, 3000)
    I, J = np.minimum(I, J), np.maximum(I, J)
    I = np.concatenate([I, np.arange(n)])
    J = np.concatenate([J, np.arange(n)])
    ref = og.gram_entries(space, p, "trilinear", X[0], I, J)
    got = out[og.packed_offset(I, J)]
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= TOL64 * scale
    # the packed output of one element carries no garbage: every entry finite
    assert np.isfinite(out).all()


def test_bad_element_zeroed_and_flagged(ctx, dpg):
    say("bad element")
    X = meshgen.perturbed_hexes(3, seed=5)
    X[1][[0, 7]] = X[1][[7, 0]]
    st = torch.full((3,), 99, dtype=torch.int32, device="cuda")
    for space in SPACES:
        out = run(ctx, space, 3, X, status=st).cpu().numpy()
        s = st.cpu().numpy()
        assert list(s) == [0, dpg.EJACOBIAN, 0]
        m = dpg.packed_len(space, 3)
        assert np.all(out[m:2 * m] == 0)
        compare64(elem(out, 0, space, 3), og.gram(space, 3, "trilinear", X[0]), "neighbour 0")
        compare64(elem(out, 2, space, 3), og.gram(space, 3, "trilinear", X[2]), "neighbour 2")


def test_empty_and_invalid(ctx, dpg):
    say("empty / invalid")
    g = torch.zeros((0, 8, 3), dtype=torch.float64, device="cuda")
    out = ctx.gram("H1", 3, g)
    assert out.numel() == 0
    X = torch.from_numpy(meshgen.perturbed_hexes(1)).cuda()
    with pytest.raises(dpg.DpgError):
        ctx.gram("H1", 12, X)
    with pytest.raises(dpg.DpgError):
        ctx.gram("H1", 3, X, nq=12)                      # more points than any built rule
    with pytest.raises(dpg.DpgError):
        ctx.gram("H1", 11, X, nq=11)                     # other rules up to p = 10 only
    with pytest.raises(dpg.DpgError):
        ctx.gram("H1", 3, X, path="reduced")
    A = torch.from_numpy(meshgen.affine_parallelepipeds(1, seed=2)).cuda()
    with pytest.raises(dpg.DpgError):
        ctx.gram("H1", 3, A, kind="affine", path="reduced", nq=6)   # the reduced path takes no rule


def test_config2_full_size_sampled(ctx, dpg):
    """4096 distorted hexes, H1 p=7: the benchmark launch; sampled elements vs oracle."""
    say("config 2 full size fp64 + fp32")
    X = meshgen.perturbed_hexes(4096, seed=1712)
    g = torch.from_numpy(X).cuda()
    m = dpg.packed_len("H1", 7)
    out = ctx.gram("H1", 7, g)
    out32 = ctx.gram("H1", 7, g, prec="fp32")
    torch.cuda.synchronize()
    for e in (0, 1, 2047, 4095):
        R = og.gram("H1", 7, "trilinear", X[e])
        G = og.unpack_upper(out[e * m:(e + 1) * m].cpu().numpy(), 512)
        compare64(G, R, f"config2 e={e}")
        G32 = og.unpack_upper(out32[e * m:(e + 1) * m].cpu().numpy().astype(np.float64), 512)
        fro = np.linalg.norm(G32 - R) / np.linalg.norm(R)
        say(f"  config2 fp32 e={e} rel fro {fro:.3e}")
        assert fro <= FP32_REL
    # whole-batch property: every diagonal entry positive, every entry finite
    diag = torch.arange(512, device="cuda")
    doff = diag * (diag + 1) // 2 + diag
    D = out.view(4096, m)[:, doff]
    assert bool(torch.isfinite(out).all()) and bool((D > 0).all())


@pytest.mark.parametrize("space", ["HCURL", "HDIV"])
def test_config3_affine_sampled(ctx, dpg, space):
    say(f"config 3 {space}")
    for p, E in ((4, 20000), (6, 2000), (8, 400)):
        A = meshgen.affine_parallelepipeds(E, seed=1713)
        g = torch.from_numpy(A).cuda()
        m = dpg.packed_len(space, p)
        n = dpg.gram_dim(space, p)
        red = ctx.gram(space, p, g, kind="affine", path="reduced")
        gen = ctx.gram(space, p, g, kind="affine", path="general")
        torch.cuda.synchronize()
        for e in (0, E - 1):
            R = og.gram(space, p, "affine", A[e])
            compare64(og.unpack_upper(red[e * m:(e + 1) * m].cpu().numpy(), n), R, f"reduced {space} p={p}")
            compare64(og.unpack_upper(gen[e * m:(e + 1) * m].cpu().numpy(), n), R, f"general {space} p={p}")
        d = (red - gen).abs().max().item() / red.abs().max().item()
        say(f"  {space} p={p} E={E} reduced vs general max rel {d:.2e}")
        assert d <= TOL64
        del red, gen
        torch.cuda.empty_cache()


def test_batched_equals_single(ctx, dpg):
    say("batched uneven p")
    space, pr, X = meshgen.mixed_batch(300, p_lo=2, p_hi=9, dp=1, seed=1714)
    lens = np.array([dpg.packed_len(int(s), int(p)) for s, p in zip(space, pr)])
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    total = int(lens.sum())
    for prec, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        out = torch.full((total,), float("nan"), dtype=dt, device="cuda")
        ctx.gram_batched(torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda(),
                         torch.from_numpy(X).cuda(), torch.from_numpy(off).cuda(), out, prec=prec)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(out).all())
        for e in range(0, 300, 7):
            s, p = int(space[e]), int(pr[e])
            single = ctx.gram(s, p, torch.from_numpy(X[e:e + 1]).cuda(), prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(out[off[e]:off[e] + lens[e]], single), (e, s, p)
        for e in (0, 1):
            s, p = int(space[e]), int(pr[e])
            name = SPACES[s]
            n = dpg.gram_dim(s, p)
            G = og.unpack_upper(out[off[e]:off[e] + lens[e]].cpu().numpy().astype(np.float64), n)
            R = og.gram(name, p, "trilinear", X[e])
            if prec == "fp64":
                compare64(G, R, f"batched {name} p={p}")


def test_batched_host_arrays_equal_device_arrays(ctx, dpg):
    """dpg_gram_integrate_batched_host (space/p on the host, no read back) gives the
    batched call's matrices bit for bit, also on a replay of its cached plan and after
    the host arrays change in place (a new plan)."""
    say("batched, host space/p")
    space, pr, X = meshgen.mixed_batch(200, p_lo=1, p_hi=8, dp=1, seed=71)
    lens = np.array([dpg.packed_len(int(s), int(p)) for s, p in zip(space, pr)])
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    X_d, off_d = torch.from_numpy(X).cuda(), torch.from_numpy(off).cuda()
    ref = torch.empty(int(lens.sum()), dtype=torch.float64, device="cuda")
    ctx.gram_batched(torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda(), X_d, off_d, ref)
    got = torch.empty_like(ref)
    n0 = ctx.batch_plans()
    for rep in range(3):
        got.fill_(float("nan"))
        ctx.gram_batched_host(space, pr, X_d, off_d, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), rep
    assert ctx.batch_plans() == min(8, n0 + 1)
    sp2 = space.copy()
    pr2 = pr.copy()
    pr2[3] = 1 if pr2[3] != 1 else 2
    lens2 = np.array([dpg.packed_len(int(s), int(p)) for s, p in zip(sp2, pr2)])
    off2 = torch.from_numpy(np.concatenate([[0], np.cumsum(lens2)[:-1]]).astype(np.int64)).cuda()
    ref2 = torch.empty(int(lens2.sum()), dtype=torch.float64, device="cuda")
    got2 = torch.empty_like(ref2)
    ctx.gram_batched(torch.from_numpy(sp2).cuda(), torch.from_numpy(pr2).cuda(), X_d, off2, ref2)
    ctx.gram_batched_host(sp2, pr2, X_d, off2, got2)
    torch.cuda.synchronize()
    assert torch.equal(got2, ref2)
    with pytest.raises(dpg.DpgError):
        bad = pr.copy()
        bad[0] = 12
        ctx.gram_batched_host(space, bad, X_d, off_d, got)


def test_slab_groups_bitwise_identical_and_autotune(dpg, tmp_path):
    """Every work decomposition computes each entry with the same operation
    sequence, so outputs are bitwise equal; the tuner's choice is one of them.
    Runs on a context with an empty tuning table (not the shipped one)."""
    say("autotune / slab groups")
    ctx = dpg.Context(p_max=11, tune_table=None)
    X = torch.from_numpy(meshgen.perturbed_hexes(64, seed=3)).cuda()
    for space, p in (("H1", 5), ("HCURL", 3), ("HDIV", 4), ("L2", 5)):
        ref = ctx.gram(space, p, X)
        torch.cuda.synchronize()
        best = ctx.autotune(space, p, X)
        ns = sum(shapes.ranges(space, p)[a][2] for a in range(len(shapes.ranges(space, p))))
        assert 1 <= best <= ns
        assert ctx.tune_lookup(space, p, n_elem=64) == best
        out = ctx.gram(space, p, X)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), space
    f = tmp_path / "tune.json"
    ctx.tune_save(f)
    c2 = dpg.Context(p_max=11, tune_table=None)
    try:
        assert c2.tune_lookup("H1", 5, n_elem=64) == 0
        c2.tune_load(f)
        assert c2.tune_lookup("H1", 5, n_elem=64) == ctx.tune_lookup("H1", 5, n_elem=64)
        assert c2.tune_lookup("H1", 5, n_elem=64 * 4) == ctx.tune_lookup("H1", 5, n_elem=64)   # nearby class
        assert c2.tune_lookup("H1", 5, n_elem=64 * 1024) == 0                                 # too far
    finally:
        c2.close()
        ctx.close()


def test_batched_graph_replays(ctx, dpg):
    """The batched dispatch replays a captured graph: repeat it with eager work and
    synchronisations in between and check every replay against eager single calls."""
    say("batched graph replay")
    space, pr, X = meshgen.mixed_batch(120, p_lo=1, p_hi=6, dp=1, seed=99)
    lens = np.array([dpg.packed_len(int(s), int(p)) for s, p in zip(space, pr)])
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    sp_d, pr_d = torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda()
    X_d, off_d = torch.from_numpy(X).cuda(), torch.from_numpy(off).cuda()
    out = torch.empty(int(lens.sum()), dtype=torch.float64, device="cuda")
    eager = torch.empty_like(out)
    for e in range(120):
        eager[off[e]:off[e] + lens[e]] = ctx.gram(int(space[e]), int(pr[e]), X_d[e:e + 1])
    torch.cuda.synchronize()
    n0 = ctx.batch_plans()
    for rep in range(4):
        out.fill_(float("nan"))                      # eager work between replays
        torch.cuda.synchronize()
        ctx.gram_batched(sp_d, pr_d, X_d, off_d, out)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
    assert ctx.batch_plans() == n0 + 1               # one plan, replayed
    pr2 = pr.copy()
    pr2[0] = 1 if pr2[0] != 1 else 2                 # same pointers, new contents -> new plan
    pr_d.copy_(torch.from_numpy(pr2))
    lens2 = np.array([dpg.packed_len(int(s), int(p)) for s, p in zip(space, pr2)])
    off2 = np.concatenate([[0], np.cumsum(lens2)[:-1]]).astype(np.int64)
    off_d.copy_(torch.from_numpy(off2))
    out2 = torch.empty(int(lens2.sum()), dtype=torch.float64, device="cuda")
    ctx.gram_batched(sp_d, pr_d, X_d, off_d, out2)
    torch.cuda.synchronize()
    assert ctx.batch_plans() == n0 + 2
    single = ctx.gram(int(space[0]), int(pr2[0]), X_d[0:1])
    torch.cuda.synchronize()
    assert torch.equal(out2[:lens2[0]], single)


def _force_schedule(ctx, tmp_path, space, p, prec, n, G, diag):
    """Pin the work decomposition through the tuning table (a JSON row):
    G slabs per workgroup, diagonal pairs last (0) or closing their slab (1)."""
    import json
    sid = {"H1": 0, "HCURL": 1, "HDIV": 2, "L2": 3}[space]
    f = tmp_path / f"force_{space}_{p}_{prec}_{G}_{diag}.json"
    f.write_text(json.dumps({"arch": "gfx950", "fields": [], "tune": [
        [sid, p, 0 if prec == "fp64" else 1, 0, int(np.floor(np.log2(n))), G, 1.0, diag]]}))
    ctx.tune_load(f)


@pytest.mark.parametrize("space,p", [("H1", 7), ("L2", 8), ("HCURL", 4), ("H1", 9), ("HDIV", 6), ("HCURL", 5)])
def test_every_schedule_agrees(ctx, dpg, tmp_path, space, p):
    """Slab groups move the workgroup boundaries; the diagonal schedule moves the
    diagonal pairs between their own triangular-tile batches and the end of each
    slab (full tile, lower triangle dropped).  Every combination must give the same
    output bit for bit, and the oracle within the FP64 / FP32 tolerances (p <= 7).
    Covers two pairs per row tile (H1 7), one (L2 8, H1 9) and three-component spaces
    (H(curl) 4, 5, H(div) 6)."""
    say(f"schedules {space} p={p}")
    n = 5
    X = meshgen.perturbed_hexes(n, seed=81)
    ns = sum(r[2] for r in shapes.ranges(space, p))
    ref = {e: og.gram(space, p, "trilinear", X[e]) for e in (0, n - 1)} if p <= 7 else {}
    sampled = (0, n - 1) if p > 7 else ()
    for prec in ("fp64", "fp32"):
        outs = []
        for G in sorted({1, 2, 3, ns}):
            for diag in (0, 1):
                _force_schedule(ctx, tmp_path, space, p, prec, n, G, diag)
                assert ctx.tune_lookup(space, p, prec=prec, n_elem=n) == G
                outs.append(run(ctx, space, p, X, prec=prec).cpu().numpy())
        for o in outs[1:]:
            assert np.array_equal(o, outs[0]), f"{space} p={p} {prec}: schedules disagree"
        for e, R in ref.items():
            G_ = elem(outs[0], e, space, p)
            if prec == "fp64":
                compare64(G_, R, f"{space} p={p} element {e}")
            else:
                fro = np.linalg.norm(G_ - R) / np.linalg.norm(R)
                assert fro <= FP32_REL, f"{space} p={p} fp32 element {e}: {fro:.3e}"
        for e in sampled:
            compare_sampled(outs[0], e, space, p, "trilinear", X[e], seed=20 + e, what=f"{space} p={p} {prec} e={e}",
                            tol=TOL64 if prec == "fp64" else FP32_REL)


def test_tune_table_rows(ctx, dpg, tmp_path):
    """Tables written before the diagonal schedule existed (7 fields) still load;
    a diagonal schedule outside {-1, 0, 1} is rejected."""
    import json
    f = tmp_path / "old.json"
    f.write_text(json.dumps({"arch": "gfx950", "fields": [], "tune": [[0, 4, 0, 0, 3, 2, 1.0]]}))
    ctx.tune_load(f)
    assert ctx.tune_lookup("H1", 4, n_elem=8) == 2
    f.write_text(json.dumps({"arch": "gfx950", "fields": [], "tune": [[0, 4, 0, 0, 3, 2, 1.0, 5]]}))
    with pytest.raises(dpg.DpgError):
        ctx.tune_load(f)
