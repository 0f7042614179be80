"""The allocation-free uneven batch (dpg_gram_integrate_batched_noalloc) against
the batched call it stands in for (dpg_gram_integrate_batched), through the C ABI.

Both run the same Gram kernels on every element, so the matrices must agree
bit for bit (the integer/byte bar: exact equality).  Two calls in a row, the
second with fewer elements, so the second reads lists built over the first
call's longer ones; both precisions; trilinear and affine geometry; status
words; an element with an invalid order; the size limit.
"""
import numpy as np
import pytest
import torch

import meshgen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu noalloc]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def batch(dpg, n, seed, p_lo=1, p_hi=10):
    space, pr, X = meshgen.mixed_batch(n, p_lo=p_lo, p_hi=p_hi, dp=1, seed=seed)
    lens = np.array([dpg.packed_len(int(s), int(q)) for s, q in zip(space, pr)], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    return space, pr, X, off, int(lens.sum())


def test_noalloc_equals_batched_two_calls(ctx, dpg):
    for prec, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        for n, seed in ((400, 11), (123, 12)):       # the second call is smaller
            say(f"{prec} n={n}")
            space, pr, X, off, total = batch(dpg, n, seed)
            args = (torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda(), torch.from_numpy(X).cuda(),
                    torch.from_numpy(off).cuda())
            ref = torch.full((total,), float("nan"), dtype=dt, device="cuda")
            got = torch.full((total,), float("nan"), dtype=dt, device="cuda")
            st_ref = torch.full((n,), 99, dtype=torch.int32, device="cuda")
            st_got = torch.full((n,), 99, dtype=torch.int32, device="cuda")
            ctx.gram_batched(*args, ref, prec=prec, status=st_ref)
            ctx.gram_batched_noalloc(*args, got, prec=prec, status=st_got)
            torch.cuda.synchronize()
            assert bool(torch.isfinite(ref).all())
            assert torch.equal(got, ref), f"{prec} n={n}: outputs differ"
            assert torch.equal(st_got, st_ref) and int(st_got.abs().sum()) == 0


def test_noalloc_affine_reduced(ctx, dpg):
    say("affine geometry, reduced path")
    n = 200
    space, pr, _, off, total = batch(dpg, n, 21, p_lo=1, p_hi=8)
    A = torch.from_numpy(meshgen.affine_parallelepipeds(n, seed=22)).cuda()
    args = (torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda(), A, torch.from_numpy(off).cuda())
    ref = torch.empty(total, dtype=torch.float64, device="cuda")
    got = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.gram_batched(*args, ref, kind="affine")
    ctx.gram_batched_noalloc(*args, got, kind="affine")
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_invalid_element_and_limits(ctx, dpg):
    say("invalid element, size limit")
    n = 50
    space, pr, X, off, total = batch(dpg, n, 31, p_lo=1, p_hi=6)
    bad = 7
    pr_bad = pr.copy()
    pr_bad[bad] = 12                                   # above p_max: skipped, flagged
    args = (torch.from_numpy(space).cuda(), torch.from_numpy(pr_bad).cuda(), torch.from_numpy(X).cuda(),
            torch.from_numpy(off).cuda())
    got = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    ctx.gram_batched_noalloc(*args, got, status=st)
    ref = torch.empty(total, dtype=torch.float64, device="cuda")
    ctx.gram_batched(torch.from_numpy(space).cuda(), torch.from_numpy(pr).cuda(), torch.from_numpy(X).cuda(),
                     torch.from_numpy(off).cuda(), ref)
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    assert s[bad] == dpg.EINVAL and (np.delete(s, bad) == 0).all()
    m = dpg.packed_len(int(space[bad]), int(pr[bad]))
    lo = int(off[bad])
    assert bool(torch.isnan(got[lo:lo + m]).all())     # untouched
    keep = torch.ones(total, dtype=torch.bool, device="cuda")
    keep[lo:lo + m] = False
    assert torch.equal(got[keep], ref[keep])
    # more elements than the list array holds: rejected before any device work
    big = dpg.noalloc_max_elements() + 1
    g = torch.zeros(big * 24, dtype=torch.float64, device="cuda")
    sp = torch.zeros(big, dtype=torch.int8, device="cuda")
    o = torch.zeros(big, dtype=torch.int64, device="cuda")
    with pytest.raises(dpg.DpgError) as ei:
        ctx.gram_batched_noalloc(sp, sp, g, o, g)
    assert ei.value.code == dpg.EINVAL
    # empty batch: nothing to do
    z8 = torch.zeros(0, dtype=torch.int8, device="cuda")
    ctx.gram_batched_noalloc(z8, z8, torch.zeros(0, dtype=torch.float64, device="cuda"),
                             torch.zeros(0, dtype=torch.int64, device="cuda"),
                             torch.zeros(0, dtype=torch.float64, device="cuda"))
