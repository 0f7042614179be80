"""GPU parity of the adjoint-graph coupling block (Section 3.3, (3.17), (3.18))
and of the block-diagonal replication for vector-valued spaces (Section 2.7,
(2.85)-(2.88)), through the C ABI.

Tolerances: coupling FP64 1e-12 and FP32 2e-6 relative to max |C| (the GPU
evaluates the exact product formula, the oracle a quadrature of the physical
fields: both are exact up to rounding); replication is a copy, compared bit for
bit with numpy's block-diagonal expansion of the same Grams, and against the
oracle's product-space Gram within 1e-12.
"""
import numpy as np
import pytest
import torch

import meshgen
from oracle import adjoint
from oracle import gram as og
from oracle import shapes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-adjoint]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 9])
def test_coupling_vs_oracle(ctx, p):
    say("coupling", p)
    R = adjoint.coupling(p)
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-6)):
        C = ctx.adjoint_coupling(p, prec=prec)
        torch.cuda.synchronize()
        C = C.cpu().numpy().astype(np.float64)
        assert C.shape == R.shape
        err = np.abs(C - R).max() / np.abs(R).max()
        assert err <= tol, f"p={p} {prec}: {err:.3e}"


def test_coupling_is_element_independent_on_the_gpu_too(ctx):
    """The same C serves every element: compare with the oracle on a distorted element."""
    p = 3
    X = meshgen.perturbed_hexes(1, noise=0.2, seed=240)[0]
    R = adjoint.coupling(p, "trilinear", X)
    C = ctx.adjoint_coupling(p).cpu().numpy()
    assert np.abs(C - R).max() <= 1e-12 * np.abs(R).max()


def _expand(ap, n, copies):
    G = og.unpack_upper(ap, n)
    return og.packed_upper(np.kron(np.eye(copies), G))


@pytest.mark.parametrize("space,p", [("H1", 3), ("HDIV", 2), ("HCURL", 3), ("L2", 4)])
def test_replicate_blocks(ctx, dpg, space, p):
    say("replicate", space, p)
    n = dpg.gram_dim(space, p)
    m = n * (n + 1) // 2
    X = meshgen.perturbed_hexes(5, seed=250)                  # ragged count
    g = torch.from_numpy(X).cuda()
    for prec in ("fp64", "fp32"):
        G = ctx.gram(space, p, g, prec=prec)
        torch.cuda.synchronize()
        Gn = G.cpu().numpy()
        for copies in (1, 2, 3):
            out = ctx.replicate_blocks(G, n, copies, prec=prec)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            cm = (copies * n) * (copies * n + 1) // 2
            assert o.size == 5 * cm
            for e in range(5):
                ref = _expand(Gn[e * m:(e + 1) * m].astype(np.float64), n, copies).astype(o.dtype)
                assert np.array_equal(o[e * cm:(e + 1) * cm], ref), (space, p, prec, copies, e)
    # against the oracle's product-space Gram (FP64)
    out = ctx.replicate_blocks(ctx.gram(space, p, g), n, 3).cpu().numpy()
    cm = (3 * n) * (3 * n + 1) // 2
    V = og.vector_gram(space, p, "trilinear", X[1], 3)
    Vg = og.unpack_upper(out[cm:2 * cm], 3 * n)
    assert np.abs(Vg - V).max() <= 1e-12 * np.abs(V).max()


def test_replicate_errors(ctx, dpg):
    n = dpg.gram_dim("H1", 2)
    m = n * (n + 1) // 2
    src = torch.zeros(2 * m, dtype=torch.float64, device="cuda")
    for copies in (0, 5):
        with pytest.raises(dpg.DpgError):
            ctx.replicate_blocks(src, n, copies)
    big = torch.zeros(2 * (3 * n) * (3 * n + 1) // 2, dtype=torch.float64, device="cuda")
    with pytest.raises(dpg.DpgError):                          # destination overlaps the source
        ctx.replicate_blocks(big[:2 * m], n, 3, out=big)
    with pytest.raises(dpg.DpgError):
        ctx.adjoint_coupling(0)
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert ctx.replicate_blocks(empty, n, 3).numel() == 0
