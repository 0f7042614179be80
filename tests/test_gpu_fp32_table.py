"""FP32 path error table: per space and order p, the relative Frobenius error
of the FP32 Gram matrices against the FP64 oracle, and whether each FP32 Gram
passes a single-precision Cholesky factorisation.

Reference: the oracle itself for every row.  Where the full oracle matrix is
cheap (n <= 350) the error is over the whole matrix; above that it is over a
sample of entries computed one by one (og.gram_entries): the whole diagonal
plus 3000 random upper-triangle entries, which carries most of the matrix
norm.  The table is written to gpurun_out/fp32_error_table.json when that
folder exists.  Bound asserted: FP32_TABLE_BOUND = twice the largest error
measured over all rows, on every element.
"""
import json
import os

import numpy as np
import pytest
import torch

import meshgen
from oracle import gram as og
from oracle import shapes

pytestmark = pytest.mark.gpu

SPACES = ["H1", "HCURL", "HDIV", "L2"]
FP32_TABLE_BOUND = 5e-7
N_ELEM = 3
FULL_MAX_N = 350


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def unpack(flat, e, n):
    m = n * (n + 1) // 2
    return og.unpack_upper(flat[e * m:(e + 1) * m].astype(np.float64), n)


def chol_ok(G, dtype):
    try:
        np.linalg.cholesky(G.astype(dtype))
        return True
    except np.linalg.LinAlgError:
        return False


def sample(n, seed, k=3000):
    rng = np.random.default_rng(seed)
    I = rng.integers(0, n, k)
    J = rng.integers(0, n, k)
    I, J = np.minimum(I, J), np.maximum(I, J)
    return np.concatenate([I, np.arange(n)]), np.concatenate([J, np.arange(n)])


def test_fp32_error_table(ctx, dpg):
    X = meshgen.perturbed_hexes(N_ELEM, noise=0.15, seed=1712)
    g = torch.from_numpy(X).cuda()
    rows = []
    worst = 0.0
    for space in SPACES:
        for p in range(1, 12):
            print(f"[fp32 table] {space} p={p}", flush=True)
            n = shapes.dimension(space, p)
            m = n * (n + 1) // 2
            o64 = ctx.gram(space, p, g, prec="fp64").cpu().numpy()
            o32 = ctx.gram(space, p, g, prec="fp32").cpu().numpy()
            errs, errs64 = [], []
            for e in range(N_ELEM):
                if n <= FULL_MAX_N:
                    R = og.gram(space, p, "trilinear", X[e])
                    G32, G64 = unpack(o32, e, n), unpack(o64, e, n)
                else:
                    I, J = sample(n, seed=e)
                    R = og.gram_entries(space, p, "trilinear", X[e], I, J)
                    off = og.packed_offset(I, J)
                    G32 = o32[e * m:(e + 1) * m][off].astype(np.float64)
                    G64 = o64[e * m:(e + 1) * m][off]
                errs.append(float(np.linalg.norm(G32 - R) / np.linalg.norm(R)))
                errs64.append(float(np.linalg.norm(G64 - R) / np.linalg.norm(R)))
            G32 = unpack(o32, 0, n)
            G64 = unpack(o64, 0, n)
            ev = np.linalg.eigvalsh(G64)
            rows.append(dict(space=space, p=p, dim=n, max_rel_fro=max(errs), mean_rel_fro=float(np.mean(errs)),
                             fp64_max_rel_fro=max(errs64),
                             cond_fp64=float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf"),
                             cholesky_fp32=chol_ok(G32, np.float32), cholesky_fp64=chol_ok(G64, np.float64),
                             reference="oracle, full matrix" if n <= FULL_MAX_N else "oracle, diagonal + 3000 entries"))
            worst = max(worst, max(errs))
            assert max(errs64) <= 1e-12, rows[-1]
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "fp32_error_table.json"), "w") as fh:
            json.dump(rows, fh, indent=1)
    for r in rows:
        print(json.dumps(r), flush=True)
    print(f"[fp32 table] worst {worst:.3e}", flush=True)
    assert all(r["cholesky_fp64"] for r in rows)
    assert worst <= FP32_TABLE_BOUND, f"worst FP32 relative Frobenius error {worst:.3e}"
