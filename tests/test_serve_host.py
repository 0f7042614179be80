"""Host-side tests of the serving scheduler (no GPU).

The server runs with its timing stub (test_executor=True): the stub computes
nothing and finishes each launch after test_launch_s + bytes/test_bytes_per_s,
one FIFO per stream, so admission, merging, overlap, cancellation, failure
handling and the latency statistics are exercised exactly as on the device.
"""
import threading
import time

import numpy as np
import pytest

from tests._lib import load_binding

dpg = load_binding()


def geom(n, kind="trilinear"):
    return np.zeros(n * {"trilinear": 24, "affine": 12, "extruded": 10}[kind])


def req_bytes(space, pr, n, prec="fp64"):
    return n * dpg.packed_len(space, pr) * (8 if prec == "fp64" else 4)


def drain(s, tickets, release=True, timeout=10.0):
    """Poll until every ticket finished; returns {ticket: result}."""
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = s.poll(t)
            if r is not None:
                out[t] = r
                if release:
                    s.release(t)
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.0005)
    return out


def test_single_request_lifecycle():
    s = dpg.Server(None, test_executor=True)
    t = s.submit("H1", 3, geom(64), dp=1)
    r = drain(s, [t], release=False)[t]
    assert r["status"] == dpg.OK and r["p"] == 4 and r["n_elem"] == 64
    assert r["packed_len"] == dpg.packed_len("H1", 4) and r["out"] is None   # the stub has no memory
    assert 0 <= r["t_submit"] <= r["t_admit"] <= r["t_done"]
    st = s.stats()
    assert st["completed"] == 1 and st["elements"] == 64 and st["admitted_bytes"] >= req_bytes("H1", 4, 64)
    s.release(t)
    assert s.stats()["admitted_bytes"] == 0
    with pytest.raises(dpg.DpgError):
        s.poll(t)                     # released tickets are gone
    s.close()


def test_admission_respects_budget_and_fifo():
    n, sp, pr = 256, "HCURL", 5
    b = req_bytes(sp, pr, n)
    budget = 3 * (b + 256)
    s = dpg.Server(None, mem_budget_bytes=budget, test_executor=True, test_bytes_per_s=b / 0.004)
    tickets = [s.submit(sp, pr, geom(n)) for _ in range(12)]
    seen_inflight = []
    res, t0 = {}, time.time()
    while len(res) < len(tickets):
        st = s.stats()
        seen_inflight.append(st["inflight"])
        assert st["admitted_bytes"] <= budget
        for t in tickets:
            if t not in res:
                r = s.poll(t)
                if r is not None:
                    res[t] = r
                    s.release(t)
        assert time.time() - t0 < 10
        time.sleep(0.0005)
    st = s.stats()
    assert st["peak_admitted_bytes"] <= budget and st["completed"] == 12
    assert max(seen_inflight) <= 3
    admits = [res[t]["t_admit"] for t in tickets]
    assert admits == sorted(admits), "admission is first come, first served"
    s.close()


def test_continuous_batching_overlaps_running_work():
    # a long request is on the device; a short one arriving later is admitted
    # and finishes while the long one still runs (two streams)
    s = dpg.Server(None, test_executor=True, n_streams=2, test_bytes_per_s=1e9)
    big = s.submit("HDIV", 6, geom(64))             # ~0.1 s on the stub
    time.sleep(0.01)
    small = s.submit("L2", 2, geom(64))
    res = drain(s, [big, small])
    assert res[small]["t_admit"] < res[big]["t_done"]
    assert res[small]["t_done"] < res[big]["t_done"]
    assert s.stats()["max_concurrent_launches"] == 2
    s.close()


def test_same_key_requests_admitted_together_share_one_launch():
    n = 64
    b = req_bytes("H1", 5, n)
    s = dpg.Server(None, mem_budget_bytes=4 * (b + 256), test_executor=True)
    blocker = s.submit("H1", 5, geom(4 * n))          # takes the whole budget
    drain(s, [blocker], release=False)
    small = [s.submit("H1", 5, geom(n)) for _ in range(4)]
    time.sleep(0.01)
    assert s.stats()["queued"] == 4                   # waiting for memory
    s.release(blocker)                                # frees the budget: all four fit at once
    res = drain(s, small)
    st = s.stats()
    assert st["launches"] == 2 and st["completed"] == 5
    assert len({res[t]["t_admit"] for t in small}) == 1
    s.close()


def test_max_merge_and_keys_split_launches():
    n = 64
    b = req_bytes("H1", 5, n)
    s = dpg.Server(None, mem_budget_bytes=6 * (b + 256), max_merge=2, test_executor=True)
    blocker = s.submit("H1", 5, geom(6 * n))
    drain(s, [blocker], release=False)
    small = [s.submit("H1", 5, geom(n)) for _ in range(3)] + [s.submit("H1", 5, geom(n), prec="fp32")]
    time.sleep(0.01)
    s.release(blocker)
    drain(s, small)
    # 3 fp64 requests with max_merge 2 -> 2 launches; the fp32 one has another key -> 1 launch
    assert s.stats()["launches"] == 1 + 2 + 1
    s.close()


def test_max_inflight():
    s = dpg.Server(None, max_inflight=2, test_executor=True, test_bytes_per_s=1e9)
    tickets = [s.submit("L2", 6, geom(128)) for _ in range(6)]
    peak, res = 0, {}
    t0 = time.time()
    while len(res) < 6:
        peak = max(peak, s.stats()["inflight"])
        for t in tickets:
            if t not in res and (r := s.poll(t)) is not None:
                res[t] = r
                s.release(t)
        assert time.time() - t0 < 10
    assert peak <= 2
    s.close()


def test_queue_full_gives_eagain():
    n = 64
    s = dpg.Server(None, mem_budget_bytes=req_bytes("H1", 3, n) + 256, max_queue=2, test_executor=True)
    a = s.submit("H1", 3, geom(n))
    drain(s, [a], release=False)                      # holds the whole budget
    q1, q2 = s.submit("H1", 3, geom(n)), s.submit("H1", 3, geom(n))
    with pytest.raises(dpg.DpgError) as e:
        s.submit("H1", 3, geom(n))
    assert e.value.code == dpg.EAGAIN and "queue full" in str(e.value)
    s.release(q2)                                     # cancel a queued request
    q3 = s.submit("H1", 3, geom(n))
    assert s.stats()["rejected"] == 1 and s.stats()["cancelled"] == 1
    s.release(a)
    drain(s, [q1, q3])
    s.close()


def test_slots_exhausted_gives_eagain():
    n = 64
    s = dpg.Server(None, mem_budget_bytes=req_bytes("H1", 3, n) + 256, max_slots=3 * n, test_executor=True)
    a = s.submit("H1", 3, geom(n))
    drain(s, [a], release=False)
    q1, q2 = s.submit("H1", 3, geom(n)), s.submit("H1", 3, geom(n))   # all 3n slots in use
    with pytest.raises(dpg.DpgError) as e:
        s.submit("H1", 3, geom(1))
    assert e.value.code == dpg.EAGAIN and "slots" in str(e.value)
    s.release(q1)                                     # cancelling returns its slots
    q3 = s.submit("H1", 3, geom(n))
    s.release(a)
    drain(s, [q2, q3])
    assert s.stats()["rejected"] == 1
    s.close()


def test_invalid_requests_rejected_at_submit():
    s = dpg.Server(None, mem_budget_bytes=1 << 20, max_slots=1000, test_executor=True)
    bad = [
        dict(space=7, p=3, geom=geom(1)),
        dict(space="H1", p=0, geom=geom(1)),
        dict(space="H1", p=11, dp=1, geom=geom(1)),           # Gram order 12 > 11
        dict(space="H1", p=3, dp=-1, geom=geom(1)),
        dict(space="H1", p=3, geom=geom(1), prec=5),
        dict(space="H1", p=3, geom=geom(1), path=9),
        dict(space="H1", p=3, geom=geom(1), path="reduced"),   # reduced needs affine or extruded geometry
        dict(space="H1", p=3, geom=geom(1), kind=3),            # unknown geometry kind
        dict(space="H1", p=3, geom=geom(1), w0=float("nan")),
        dict(space="HCURL", p=8, geom=geom(4)),                # output > 1 MiB budget: split it
        dict(space="L2", p=2, geom=geom(1001)),                # more elements than slots
        dict(space="H1", p=3, geom=np.zeros(0)),
    ]
    for b in bad:
        with pytest.raises(dpg.DpgError) as e:
            s.submit(**b)
        assert e.value.code == dpg.EINVAL, b
    with pytest.raises(ValueError):
        s.submit("H1", 3, np.zeros(25))
    assert s.stats()["rejected"] == len(bad) and s.stats()["submitted"] == 0
    s.close()


def test_extruded_requests_accepted():
    """Extruded geometry (10 doubles per element) is served by either path."""
    s = dpg.Server(None, mem_budget_bytes=1 << 26, max_slots=1000, test_executor=True)
    t = [s.submit("HDIV", 3, geom(5, "extruded"), kind="extruded"),
         s.submit("HDIV", 3, geom(5, "extruded"), kind="extruded", path="general")]
    res = drain(s, t)
    assert all(r["status"] == dpg.OK and r["n_elem"] == 5 for r in res.values())
    s.close()


def test_release_of_running_request_is_refused():
    s = dpg.Server(None, test_executor=True, test_bytes_per_s=1e8)
    t = s.submit("HDIV", 5, geom(64))
    time.sleep(0.005)
    assert s.poll(t) is None
    with pytest.raises(dpg.DpgError) as e:
        s.release(t)
    assert e.value.code == dpg.EAGAIN
    drain(s, [t])
    s.close()


def test_failed_launch_surfaces_per_request_and_others_complete():
    s = dpg.Server(None, test_executor=True, test_fail_launch=2, max_merge=1)
    tickets = []
    for i in range(5):
        tickets.append(s.submit("H1", 2 + i, geom(64)))
        time.sleep(0.002)
    res = drain(s, tickets)
    status = [res[t]["status"] for t in tickets]
    assert status.count(dpg.EHIP) == 1 and status.count(dpg.OK) == 4
    st = s.stats()
    assert st["failed"] == 1 and st["completed"] == 4 and st["admitted_bytes"] == 0
    s.close()


def test_latency_statistics_match_results():
    s = dpg.Server(None, test_executor=True, test_bytes_per_s=5e10, test_launch_s=2e-4)
    rng = np.random.default_rng(3)
    tickets = []
    for _ in range(40):
        tickets.append(s.submit(int(rng.integers(4)), int(rng.integers(2, 7)), geom(int(rng.integers(64, 256)))))
        time.sleep(float(rng.exponential(0.001)))
    res = drain(s, tickets)
    lat = np.sort([res[t]["t_done"] - res[t]["t_submit"] for t in tickets])
    st = s.stats()
    nearest_rank = lambda q: lat[max(1, int(np.ceil(q * len(lat)))) - 1]
    assert st["lat_p50"] == pytest.approx(nearest_rank(0.5), abs=1e-12)
    assert st["lat_p99"] == pytest.approx(nearest_rank(0.99), abs=1e-12)
    assert st["lat_max"] == pytest.approx(lat[-1]) and st["lat_mean"] == pytest.approx(lat.mean())
    assert st["elements"] == sum(res[t]["n_elem"] for t in tickets)
    s.reset_stats()
    st = s.stats()
    assert st["completed"] == 0 and st["lat_p99"] == 0.0
    s.close()


def test_concurrent_submitters():
    s = dpg.Server(None, test_executor=True, test_bytes_per_s=1e11, max_queue=100000)
    done, errors = [], []

    def client(seed):
        rng = np.random.default_rng(seed)
        mine = []
        try:
            for _ in range(40):
                mine.append(s.submit(int(rng.integers(4)), int(rng.integers(1, 6)), geom(int(rng.integers(1, 64)))))
            done.append(len(drain(s, mine)))
        except Exception as e:    # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=client, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors and done == [40] * 4
    st = s.stats()
    assert st["completed"] == 160 and st["queued"] == 0 and st["inflight"] == 0 and st["admitted_bytes"] == 0
    s.close()


def test_destroy_with_unreleased_and_queued_requests():
    n = 64
    s = dpg.Server(None, mem_budget_bytes=req_bytes("H1", 4, n) + 256, test_executor=True, test_bytes_per_s=1e9)
    a = s.submit("H1", 4, geom(n))
    s.submit("H1", 4, geom(n))      # queued behind a
    drain(s, [a], release=False)
    s.close()                         # must not hang or leak


def test_bad_config():
    for kw in (dict(mem_budget_bytes=0), dict(n_streams=0), dict(n_streams=9), dict(max_merge=33),
               dict(max_inflight=0), dict(max_queue=0), dict(max_slots=0)):
        with pytest.raises(dpg.DpgError):
            dpg.Server(None, test_executor=True, **kw)
    with pytest.raises(dpg.DpgError) as e:
        dpg.Server(None)               # the device executor needs a context
    assert e.value.code == dpg.ENOTINIT


def test_chunked_request_streams_through_a_small_budget():
    """A request three and a half budgets large is cut into element chunks that fit
    the budget; the chunks have consecutive tickets, cover the request in order,
    and stream through as the client releases each one."""
    per = req_bytes("HCURL", 6, 1)
    budget = 100 * per + 1000
    s = dpg.Server(None, test_executor=True, mem_budget_bytes=budget, test_bytes_per_s=1e13)
    n = 350
    first, k, ce = s.submit_chunked("HCURL", 5, geom(n), dp=1)
    assert ce == budget // per == 100 and k == 4
    got = drain(s, list(range(first, first + k)))
    assert [got[first + i]["n_elem"] for i in range(k)] == [100, 100, 100, 50]
    assert all(r["status"] == dpg.OK and r["p"] == 6 for r in got.values())
    st = s.stats()
    assert st["completed"] == 4 and st["elements"] == n and st["peak_admitted_bytes"] <= budget
    # a smaller chunk size than the budget, and a request that fits one chunk
    first, k, ce = s.submit_chunked("HCURL", 5, geom(n), dp=1, max_chunk_bytes=40 * per)
    assert (k, ce) == (9, 40)
    drain(s, list(range(first, first + k)))
    first, k, ce = s.submit_chunked("L2", 3, geom(10), dp=1)
    assert k == 1 and ce >= 10
    drain(s, [first])
    s.close()


def test_chunked_request_all_or_none():
    per = req_bytes("H1", 4, 1)
    s = dpg.Server(None, test_executor=True, mem_budget_bytes=10 * per + 1024, max_queue=5, test_launch_s=0.05)
    with pytest.raises(dpg.DpgError) as e:                       # more chunks than the queue ever holds
        s.submit_chunked("H1", 3, geom(60), dp=1)
    assert e.value.code == dpg.EINVAL
    with pytest.raises(dpg.DpgError) as e:                       # one element larger than the chunk size
        s.submit_chunked("H1", 3, geom(5), dp=1, max_chunk_bytes=per // 2)
    assert e.value.code == dpg.EINVAL
    busy = [s.submit("H1", 3, geom(10), dp=1) for _ in range(3)]   # the head runs, two wait
    t0 = time.time()
    while s.stats()["admitted"] < 1 and time.time() - t0 < 10:  # the scheduler thread admits the head
        time.sleep(0.001)
    with pytest.raises(dpg.DpgError) as e:                       # 4 chunks, 3 free queue entries at most
        s.submit_chunked("H1", 3, geom(40), dp=1)
    assert e.value.code == dpg.EAGAIN
    assert s.stats()["queued"] <= 2                              # nothing of the rejected request was queued
    drain(s, busy)
    first, k, _ = s.submit_chunked("H1", 3, geom(40), dp=1)
    assert k == 4
    drain(s, list(range(first, first + k)))
    s.close()


def test_non_uniform_orders():
    """Requests of non-uniform orders (p1, p2, p3): sized by the per-direction Gram
    orders, merged only with requests of the same orders, validated like the
    entry point (orders in [1, 10], no reduced path)."""
    s = dpg.Server(None, test_executor=True, test_launch_s=0.002)
    t = s.submit("HCURL", (3, 2, 1), geom(20), dp=1)                # Gram orders (4, 3, 2)
    r = drain(s, [t], release=False)[t]
    nd = dpg.gram_dim_aniso("HCURL", (4, 3, 2))
    assert r["status"] == dpg.OK and r["p"] == 4 and r["n_elem"] == 20 and r["packed_len"] == nd * (nd + 1) // 2
    s.release(t)
    s.reset_stats()
    # same orders merge; different orders, or the uniform order, do not
    ts = [s.submit("H1", (5, 4, 3), geom(10)) for _ in range(3)] + [s.submit("H1", (5, 4, 2), geom(10)),
                                                                      s.submit("H1", 5, geom(10))]
    drain(s, ts)
    assert 3 <= s.stats()["launches"] <= 5
    for bad in ((0, 2, 3), (1, 2, -1), (10, 2, 2)):
        with pytest.raises(dpg.DpgError) as e:                      # dp = 1: Gram order 11 > 10
            s.submit("H1", bad, geom(4), dp=1)
        assert e.value.code == dpg.EINVAL
    with pytest.raises(dpg.DpgError):
        s.submit("H1", (2, 3, 4), geom(4, "affine"), kind="affine", path="reduced")
    s.close()
