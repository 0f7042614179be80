"""FP32 path error table: per space and order p, the relative Frobenius error
of the FP32 Gram matrices against FP64, and whether each FP32 Gram passes a
single-precision Cholesky factorisation.

For p <= 4 the FP64 reference is the oracle itself; above that the oracle's
O(p^9) cost is replaced by the library's FP64 path, which the parity tests pin
to the oracle within 1e-12 (far below the FP32 errors measured here).  The
table is written to gpurun_out/fp32_error_table.json when that folder exists.
Bound asserted: FP32_TABLE_BOUND on every sampled element.
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
FP32_TABLE_BOUND = 1e-5
N_ELEM = 6


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


def test_fp32_error_table(ctx, dpg):
    X = meshgen.perturbed_hexes(N_ELEM, noise=0.15, seed=1712)
    g = torch.from_numpy(X).cuda()
    rows = []
    worst = 0.0
    for space in SPACES:
        for p in range(1, 12):
            print(f"[fp32 table] {space} p={p}", flush=True)
            n = shapes.dimension(space, p)
            o64 = ctx.gram(space, p, g, prec="fp64").cpu().numpy()
            o32 = ctx.gram(space, p, g, prec="fp32").cpu().numpy()
            errs = []
            for e in range(N_ELEM):
                R = og.gram(space, p, "trilinear", X[e]) if p <= 4 else unpack(o64, e, n)
                G = unpack(o32, e, n)
                errs.append(float(np.linalg.norm(G - R) / np.linalg.norm(R)))
            G32 = unpack(o32, 0, n)
            G64 = unpack(o64, 0, n)
            ev = np.linalg.eigvalsh(G64)
            rows.append(dict(space=space, p=p, dim=n, max_rel_fro=max(errs), mean_rel_fro=float(np.mean(errs)),
                             cond_fp64=float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf"),
                             cholesky_fp32=chol_ok(G32, np.float32), cholesky_fp64=chol_ok(G64, np.float64),
                             reference="oracle" if p <= 4 else "fp64 path"))
            worst = max(worst, max(errs))
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "fp32_error_table.json"), "w") as fh:
            json.dump(rows, fh, indent=1)
    for r in rows:
        print(json.dumps(r), flush=True)
    assert all(r["cholesky_fp64"] for r in rows)
    assert worst <= FP32_TABLE_BOUND, f"worst FP32 relative Frobenius error {worst:.3e}"
