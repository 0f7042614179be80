"""GPU parity of the extruded-element path (Section 2.8.1, second form of (2.89),
Algorithm 11 and its extension to H1, H(curl), H(div)) through the C ABI.

An extruded element is a trilinear map whose x1 is lambda1 xi1 + x1_0 and whose
(x2, x3) do not depend on xi1, so the oracle integrates it as that trilinear
element: its xi1 integrands are polynomials of degree <= 2p + 1, which the
L-point Gauss rule integrates exactly, so the oracle and the exact 1D integrals
F^{rs} of the reduced path agree up to rounding.  Tolerances as in
test_gpu_parity: FP64 1e-12 (relative Frobenius and max), FP32 2e-6.
"""
import json

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
    print("[gpu-extruded]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def run(ctx, space, p, E, prec="fp64", path="auto", status=None, kind="extruded"):
    g = torch.from_numpy(np.ascontiguousarray(E)).cuda()
    out = ctx.gram(space, p, g, kind=kind, prec=prec, path=path, status=status)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def elem(out_np, e, space, p):
    n = shapes.dimension(space, p)
    m = n * (n + 1) // 2
    return og.unpack_upper(out_np[e * m:(e + 1) * m].astype(np.float64), n)


def rel(G, R):
    return np.linalg.norm(G - R) / np.linalg.norm(R), np.abs(G - R).max() / np.abs(R).max()


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_extruded_vs_oracle(ctx, space, p):
    say(space, p)
    n = 5                                        # ragged: not a multiple of anything
    E = meshgen.extruded_prisms(n, seed=40 + p)
    X = meshgen.extruded_as_trilinear(E)
    o64 = run(ctx, space, p, E)
    o32 = run(ctx, space, p, E, prec="fp32")
    for e in (0, 2, n - 1):
        R = og.gram(space, p, "trilinear", X[e])
        fro, mx = rel(elem(o64, e, space, p), R)
        assert fro <= TOL64 and mx <= TOL64, f"{space} p={p} e={e}: fro {fro:.3e} max {mx:.3e}"
        fro32, _ = rel(elem(o32, e, space, p), R)
        assert fro32 <= FP32_REL, f"{space} p={p} e={e} fp32: {fro32:.3e}"


@pytest.mark.parametrize("space,p", [("H1", 7), ("HCURL", 6), ("HDIV", 8), ("L2", 11), ("H1", 11), ("HCURL", 11)])
def test_extruded_vs_general_path(ctx, space, p):
    """The O(p^6) path against the O(p^7) general path on the same extruded
    elements, given both as extruded geometry and as trilinear vertices."""
    say("vs general", space, p)
    n = 3
    E = meshgen.extruded_prisms(n, seed=60 + p)
    red = run(ctx, space, p, E)
    gen = run(ctx, space, p, E, path="general")
    tri = run(ctx, space, p, meshgen.extruded_as_trilinear(E), kind="trilinear")
    for e in range(n):
        R = elem(gen, e, space, p)
        for other, what in ((red, "reduced"), (tri, "trilinear")):
            fro, mx = rel(elem(other, e, space, p), R)
            assert fro <= TOL64 and mx <= TOL64, f"{space} p={p} e={e} {what}: fro {fro:.3e} max {mx:.3e}"
    red32 = run(ctx, space, p, E, prec="fp32")
    for e in range(n):
        fro, _ = rel(elem(red32, e, space, p), elem(gen, e, space, p))
        assert fro <= FP32_REL, f"{space} p={p} e={e} fp32: {fro:.3e}"


def test_extruded_rectangle_is_affine(ctx):
    """A rectangular cross-section makes the map affine: the extruded path must
    equal the constant-Jacobian path on the same box."""
    E = np.array([[0.3, 1.7, 0.0, 0.0, 0.8, 0.0, 0.0, 1.2, 0.8, 1.2]])
    A = np.zeros((1, 12))
    A[0, :3] = [0.3, 0.0, 0.0]
    A[0, 3:] = np.diag([1.7, 0.8, 1.2]).ravel()
    for space in SPACES:
        p = 5
        G = elem(run(ctx, space, p, E), 0, space, p)
        R = elem(run(ctx, space, p, A, kind="affine"), 0, space, p)
        fro, mx = rel(G, R)
        assert fro <= TOL64 and mx <= TOL64, f"{space}: fro {fro:.3e} max {mx:.3e}"


def test_extruded_bad_element_and_empty(ctx, dpg):
    E = meshgen.extruded_prisms(4, seed=71)
    E[1, 1] = -E[1, 1]                          # lambda1 < 0: det J < 0 everywhere
    E[3, [2, 3, 4, 5]] = E[3, [4, 5, 2, 3]]     # swap two cross-section corners: folded quad
    st = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    out = run(ctx, "HDIV", 3, E, status=st)
    assert list(st.cpu().numpy()) == [0, dpg.EJACOBIAN, 0, dpg.EJACOBIAN]
    m = dpg.packed_len("HDIV", 3)
    assert np.all(out[m:2 * m] == 0) and np.all(out[3 * m:4 * m] == 0)
    R = og.gram("HDIV", 3, "trilinear", meshgen.extruded_as_trilinear(E)[2])
    fro, _ = rel(elem(out, 2, "HDIV", 3), R)
    assert fro <= TOL64
    empty = torch.empty((0,), dtype=torch.float64, device="cuda")
    assert ctx.gram("H1", 4, empty, kind="extruded").numel() == 0
    with pytest.raises(ValueError):                         # 10 doubles per element
        ctx.gram("H1", 4, torch.zeros(15, dtype=torch.float64, device="cuda"), kind="extruded")


def _force(ctx, tmp_path, space, p, prec, n, G):
    sid = SPACES.index(space)
    f = tmp_path / f"ext_{space}_{p}_{prec}_{G}.json"
    f.write_text(json.dumps({"arch": "gfx950", "fields": [], "tune": [
        [sid, p, 0 if prec == "fp64" else 1, 2, int(np.floor(np.log2(n))), G, 1.0, -1]]}))
    ctx.tune_load(f)


@pytest.mark.parametrize("space,p", [("H1", 6), ("HCURL", 4)])
def test_extruded_slab_groups_bitwise(ctx, tmp_path, space, p):
    """Every slab-group decomposition computes each entry the same way."""
    n = 6
    E = meshgen.extruded_prisms(n, seed=90)
    ns = sum(r[2] for r in shapes.ranges(space, p))
    for prec in ("fp64", "fp32"):
        outs = []
        for G in sorted({1, 2, 3, ns}):
            _force(ctx, tmp_path, space, p, prec, n, G)
            assert ctx.tune_lookup(space, p, prec=prec, reduced=2, n_elem=n) == G
            outs.append(run(ctx, space, p, E, prec=prec))
        for o in outs[1:]:
            assert np.array_equal(o, outs[0]), f"{space} p={p} {prec}"


def test_extruded_batched_equals_single(ctx, dpg):
    n = 40
    rng = np.random.default_rng(5)
    space = rng.integers(0, 4, size=n).astype(np.int8)
    pr = rng.integers(2, 9, size=n).astype(np.int8)
    E = meshgen.extruded_prisms(n, seed=91)
    lens = np.array([dpg.packed_len(int(s), int(p)) for s, p in zip(space, pr)])
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    out = torch.full((int(lens.sum()),), float("nan"), dtype=torch.float64, device="cuda")
    ctx.gram_batched(torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda(), torch.from_numpy(E).cuda(),
                     torch.from_numpy(off).cuda(), out, kind="extruded")
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    for e in range(0, n, 3):
        single = ctx.gram(int(space[e]), int(pr[e]), torch.from_numpy(E[e:e + 1]).cuda(), kind="extruded")
        torch.cuda.synchronize()
        assert torch.equal(out[off[e]:off[e] + lens[e]], single), e
