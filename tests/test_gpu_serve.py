"""GPU tests of the serving loop (dpg_serve_*), through the C ABI.

Each served result must equal the same request integrated alone
(dpg_gram_integrate on the same geometry: same kernels, so bitwise equal)
and, for orders the oracle finishes quickly, the FP64 oracle within 1e-12.
"""
import time

import numpy as np
import pytest
import torch

import meshgen
from oracle import gram as og
from oracle import shapes

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def say(*a):
    print("[gpu-serve]", *a, flush=True)


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


@pytest.fixture(scope="module")
def ctx(dpg):
    c = dpg.Context(p_max=11)
    yield c
    c.close()


def drain(srv, tickets, timeout=60.0, release=False):
    res, t0 = {}, time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res and (r := srv.poll(t)) is not None:
                res[t] = r
                if release:
                    srv.release(t)
        assert time.time() - t0 < timeout, "served requests did not finish"
        time.sleep(0.0002)
    return res


def alone(ctx, space, pr, X, kind="trilinear", prec="fp64"):
    g = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    out = ctx.gram(space, pr, g, kind=kind, prec=prec)
    torch.cuda.synchronize()
    return out


def oracle_check(out_np, e, space, pr, X, kind="trilinear"):
    n = shapes.dimension(space, pr)
    m = n * (n + 1) // 2
    G = og.unpack_upper(out_np[e * m:(e + 1) * m].astype(np.float64), n)
    R = og.gram(space, pr, kind, X[e])
    fro = np.linalg.norm(G - R) / np.linalg.norm(R)
    assert fro <= TOL64, f"{space} p={pr} element {e}: rel fro {fro:.3e}"


SPACES = ["H1", "HCURL", "HDIV", "L2"]


def test_results_same_alone_and_in_the_mix(ctx, dpg):
    say("mixed requests, alone vs served")
    rng = np.random.default_rng(2024)
    srv = dpg.Server(ctx, mem_budget_bytes=2 << 30, n_streams=4)
    reqs = []
    for i in range(16):
        space = SPACES[i % 4]
        p = int(rng.integers(1, 6))
        n = int(rng.integers(1, 300))
        X = meshgen.perturbed_hexes(n, seed=100 + i)
        prec = "fp32" if i % 5 == 4 else "fp64"
        reqs.append((space, p, 1, n, X, prec))
    tickets = [srv.submit(s, p, X.reshape(-1), dp=dp, prec=prec) for s, p, dp, n, X, prec in reqs]
    res = drain(srv, tickets)
    st = srv.stats()
    say("stats", {k: st[k] for k in ("completed", "launches", "max_concurrent_launches", "lat_p50", "lat_p99")})
    assert st["completed"] == 16 and st["failed"] == 0
    for t, (space, p, dp, n, X, prec) in zip(tickets, reqs):
        r = res[t]
        assert r["status"] == dpg.OK and r["p"] == p + dp and r["n_elem"] == n
        served = srv.read(t)
        stat = srv.read_status(t)
        torch.cuda.synchronize()
        ref = alone(ctx, space, p + dp, X, prec=prec)
        assert torch.equal(served, ref), f"{space} p={p + dp} n={n} {prec}: served != alone"
        assert int(stat.abs().sum()) == 0
        if prec == "fp64" and p + dp <= 4:
            oracle_check(served.cpu().numpy(), n - 1, space, p + dp, X)
        srv.release(t)
    assert srv.stats()["admitted_bytes"] == 0
    srv.close()


def test_merged_launch_matches_alone(ctx, dpg):
    say("merged launch")
    space, pr, n = "HDIV", 4, 100
    m = dpg.packed_len(space, pr) * 8
    srv = dpg.Server(ctx, mem_budget_bytes=4 * (n * m + 256), n_streams=2)
    Xb = meshgen.perturbed_hexes(4 * n, seed=7)
    blocker = srv.submit(space, pr, Xb.reshape(-1))          # takes the whole budget
    drain(srv, [blocker])
    geos = [meshgen.perturbed_hexes(n - 10 * k, seed=8 + k) for k in range(4)]
    small = [srv.submit(space, pr, X.reshape(-1)) for X in geos]
    time.sleep(0.02)
    assert srv.stats()["queued"] == 4
    srv.release(blocker)                                     # all four admitted in one pass -> one launch
    res = drain(srv, small)
    assert srv.stats()["launches"] == 2
    assert len({res[t]["t_admit"] for t in small}) == 1
    for t, X in zip(small, geos):
        served = srv.read(t)
        torch.cuda.synchronize()
        assert torch.equal(served, alone(ctx, space, pr, X))
    oracle_check(srv.read(small[2]).cpu().numpy(), 5, space, pr, geos[2])
    srv.close()


def test_affine_reduced_and_device_geometry(ctx, dpg):
    say("affine + device geometry")
    srv = dpg.Server(ctx, mem_budget_bytes=1 << 30)
    A = meshgen.affine_parallelepipeds(200, seed=31)
    Ad = torch.from_numpy(A.reshape(-1).copy()).cuda()
    X = meshgen.perturbed_hexes(150, seed=32)
    Xd = torch.from_numpy(X.reshape(-1).copy()).cuda()
    torch.cuda.synchronize()
    t1 = srv.submit("HCURL", 4, Ad, kind="affine")
    t2 = srv.submit("H1", 5, Xd, prec="fp32")
    t3 = srv.submit("HDIV", 3, A.reshape(-1), dp=1, kind="affine", path="general")
    drain(srv, [t1, t2, t3])
    torch.cuda.synchronize()
    assert torch.equal(srv.read(t1), alone(ctx, "HCURL", 4, A, kind="affine"))
    assert torch.equal(srv.read(t2), alone(ctx, "H1", 5, X, prec="fp32"))
    g = torch.from_numpy(A).cuda()
    ref3 = ctx.gram("HDIV", 4, g, kind="affine", path="general")
    assert torch.equal(srv.read(t3), ref3)
    oracle_check(srv.read(t1).cpu().numpy(), 17, "HCURL", 4, A, kind="affine")
    srv.close()


def test_extruded_requests_match_alone(ctx, dpg):
    say("extruded requests")
    srv = dpg.Server(ctx, mem_budget_bytes=1 << 30)
    E1 = meshgen.extruded_prisms(120, seed=51)
    E2 = meshgen.extruded_prisms(80, seed=52)
    Ed = torch.from_numpy(E2.reshape(-1).copy()).cuda()
    torch.cuda.synchronize()
    t1 = srv.submit("HCURL", 4, E1.reshape(-1), kind="extruded")               # host geometry, reduced path
    t2 = srv.submit("H1", 5, Ed, kind="extruded", prec="fp32", path="general")  # device geometry, general path
    drain(srv, [t1, t2])
    torch.cuda.synchronize()
    assert torch.equal(srv.read(t1), alone(ctx, "HCURL", 4, E1, kind="extruded"))
    g = torch.from_numpy(E2).cuda()
    assert torch.equal(srv.read(t2), ctx.gram("H1", 5, g, kind="extruded", prec="fp32", path="general"))
    oracle_check(srv.read(t1).cpu().numpy(), 7, "HCURL", 4, meshgen.extruded_as_trilinear(E1))
    srv.close()


def test_bad_element_flagged_in_served_result(ctx, dpg):
    say("bad element served")
    srv = dpg.Server(ctx, mem_budget_bytes=1 << 28)
    X = meshgen.perturbed_hexes(5, seed=41)
    X[3][[0, 7]] = X[3][[7, 0]]
    t = srv.submit("HCURL", 3, X.reshape(-1))
    ok = srv.submit("L2", 3, meshgen.perturbed_hexes(5, seed=42).reshape(-1))
    drain(srv, [t, ok])
    st = srv.read_status(t).cpu().numpy()
    assert list(st) == [0, 0, 0, dpg.EJACOBIAN, 0]
    out = srv.read(t).cpu().numpy()
    m = dpg.packed_len("HCURL", 3)
    assert np.all(out[3 * m:4 * m] == 0)
    oracle_check(out, 4, "HCURL", 3, X)
    assert list(srv.read_status(ok).cpu().numpy()) == [0] * 5
    srv.close()


def test_chunked_request_larger_than_the_budget(ctx, dpg):
    """A request four budgets large, submitted with dpg_serve_submit_chunked: the
    server cuts it into element chunks, each chunk's matrices equal the same
    elements integrated alone, bit for bit, and the chunks stream through the
    budget as the client releases them."""
    say("chunked request")
    space, pr, n = "HDIV", 6, 700
    per = dpg.packed_len(space, pr) * 8
    budget = 200 * per + 4096
    srv = dpg.Server(ctx, mem_budget_bytes=budget, max_slots=4096, n_streams=2)
    try:
        X = meshgen.perturbed_hexes(n, seed=88)
        ref = alone(ctx, space, pr, X)
        first, k, ce = srv.submit_chunked(space, pr - 1, X.reshape(-1), dp=1)
        assert ce == 200 and k == 4
        m = dpg.packed_len(space, pr)
        for c in range(k):
            t = first + c
            r = drain(srv, [t])[t]
            assert r["status"] == dpg.OK and r["n_elem"] == min(ce, n - c * ce)
            got = srv.read(t)
            torch.cuda.synchronize()
            assert torch.equal(got, ref[c * ce * m:(c * ce + r["n_elem"]) * m]), c
            srv.release(t)
        assert srv.stats()["peak_admitted_bytes"] <= budget
    finally:
        srv.close()


def test_short_poisson_trace(ctx, dpg):
    say("short Poisson trace")
    trace = meshgen.serving_trace(duration_s=0.5, rate_hz=200.0, n_lo=64, n_hi=512, p_lo=2, p_hi=6, seed=77)
    srv = dpg.Server(ctx, mem_budget_bytes=8 << 30)
    geo = [meshgen.perturbed_hexes(r["n_elem"], seed=r["seed"]).reshape(-1) for r in trace]
    t0 = time.perf_counter()
    tickets, res = [], {}
    for r, X in zip(trace, geo):
        while time.perf_counter() - t0 < r["t"]:
            pass
        tickets.append(srv.submit(r["space"], r["p"], X, dp=r["dp"]))
    keep = {t: k for k, t in enumerate(tickets) if k % 7 == 0}
    t_end = time.time() + 60
    checked = 0
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res and (x := srv.poll(t)) is not None:
                res[t] = x
                if t in keep:   # compare with the request integrated alone, then free it
                    r, X = trace[keep[t]], geo[keep[t]]
                    served = srv.read(t)
                    assert torch.equal(served, alone(ctx, r["space"], r["p"] + r["dp"], X.reshape(-1, 8, 3)))
                    checked += 1
                srv.release(t)
        assert time.time() < t_end
    st = srv.stats()
    say("trace", len(trace), "requests;", {k: st[k] for k in ("lat_p50", "lat_p99", "launches",
                                                              "max_concurrent_launches")})
    assert st["completed"] == len(trace) and st["failed"] == 0 and st["lat_p99"] >= st["lat_p50"] > 0
    assert checked == len(keep) and st["admitted_bytes"] == 0
    srv.close()


def test_non_uniform_orders_served(ctx, dpg):
    """Requests of non-uniform orders: each served result equals
    dpg_gram_integrate_aniso on the same geometry (bitwise: same kernels), the
    same-order requests in one launch, and one element against the oracle."""
    say("non-uniform orders")
    srv = dpg.Server(ctx, mem_budget_bytes=1 << 30, n_streams=2)
    cases = [("HDIV", (3, 2, 1), 1, 40), ("HDIV", (3, 2, 1), 1, 25), ("H1", (6, 5, 4), 0, 64), ("L2", (3, 4, 2), 1, 9),
             ("HCURL", (1, 1, 6), 0, 7)]                          # the last one takes the per-direction kernel
    assert ctx.aniso_route("HCURL", (1, 1, 6)) == "per-direction"
    geos = [meshgen.perturbed_hexes(n, seed=40 + k) for k, (_, _, _, n) in enumerate(cases)]
    ts = [srv.submit(sp, q, X.reshape(-1), dp=dp) for (sp, q, dp, _), X in zip(cases, geos)]
    res = drain(srv, ts)
    for t, (sp, q, dp, n), X in zip(ts, cases, geos):
        qq = tuple(x + dp for x in q)
        assert res[t]["status"] == dpg.OK and res[t]["p"] == max(qq)
        served = srv.read(t)
        a = ctx.gram_aniso(sp, qq, torch.from_numpy(X).cuda())
        torch.cuda.synchronize()
        assert torch.equal(served, a), (sp, q)
    sp, q, dp, _ = cases[2]
    nd = shapes.dimension(sp, q)
    G = og.unpack_upper(srv.read(ts[2]).cpu().numpy()[3 * nd * (nd + 1) // 2:4 * nd * (nd + 1) // 2], nd)
    R = og.gram(sp, q, "trilinear", geos[2][3])
    assert np.abs(G - R).max() / np.abs(R).max() <= TOL64
    srv.close()
