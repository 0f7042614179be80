"""Benchmark: sum-factorised DPG Gram integration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--extra | --no-extra] [--no-cpu]

One step = one dpg_gram_integrate call over the benchmark workload: 4096
trilinear hexahedra (unit-cube vertices + U(-0.15, 0.15) noise, seed 1712),
H1 test Gram of order p + dp = 7 (n = 512, 131,328 packed entries per
element), L = 8 Gauss-Legendre points per direction, FP64, general O(p^7)
path.  Inputs are resident in HBM before the timed region; outputs stay on
the device.  Prints one JSON line.

Extra measurements (FP32 path, reduced vs general affine path, uneven
batch) go into the "extra" object of the same line.  The CPU baseline times
the FP64 oracle (brute-force O(p^9) quadrature) on a bounded sample of the
same elements on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element Gram matrices/sec and % roofline at p=4..8; p50/p99 served latency"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_general_h1_p7_4096.json")
KERNEL_SOURCES = ["gram_general.inc.h", "metric.h", "terms.h", "kernels.h", "launch_limits.h", "gram_general_h1.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_00984_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind):
    """HBM bytes per launch of the benchmark kernel from the committed counter
    summary, or None if it is absent or was taken on different kernel code."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get(kind)


def time_launches(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]   # ms, on the launch stream
    return wall, per


def _oracle_worker(args):
    from threadpoolctl import threadpool_limits
    import meshgen
    from oracle import gram
    seed, idx = args
    X = meshgen.perturbed_hexes(max(idx) + 1, seed=seed)
    with threadpool_limits(1):
        t = time.perf_counter()
        for e in idx:
            gram.gram("H1", 7, "trilinear", X[e])
        return time.perf_counter() - t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(n_per_worker=1):
    """The oracle on `workers` host processes (one BLAS thread each), each
    integrating n_per_worker elements of the benchmark workload.  value = the
    elements over the slowest worker's compute time (all workers run at once);
    beside it the per-core busy rate and the wall time with the pool's start."""
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    jobs = [(1712, [w * n_per_worker + i for i in range(n_per_worker)]) for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        busy = pool.map(_oracle_worker, jobs)
        pool.close()          # let the workers exit by themselves before the block's terminate()
        pool.join()
    wall = time.perf_counter() - t0
    n = workers * n_per_worker
    return {"value": round(n / max(busy), 3), "unit": "elements/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(),
            "per_core_elements_per_s": round(n_per_worker / (sum(busy) / workers), 4),
            "wall_elements_per_s": round(n / wall, 3),
            "sample": f"{n} elements of the benchmark workload (H1, p=7, L=8), FP64 brute-force "
                      f"O(p^9) quadrature, {workers} processes x 1 BLAS thread on {cpu_model()}; "
                      f"{sum(busy):.1f} core-seconds, slowest worker {max(busy):.2f} s, "
                      f"{wall:.1f} s wall with the pool's start"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--extra", dest="extra", action="store_true", default=True)
    ap.add_argument("--no-extra", dest="extra", action="store_false")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured length of the replayed serving trace, after a 5 s warm-up "
                         "(0: skip the serving measurement)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain 4 GiB device copy (counter calibration)")
    ap.add_argument("--aniso-only", action="store_true",
                    help="run only the non-uniform-order rows (both routes)")
    ap.add_argument("--condense-only", action="store_true",
                    help="run only the condensation measurement (factor and solve of 1024 H1 p=7 Grams)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the elements are "
              "independent and the multi-GPU sharding is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    from paper_1711_00984_amd import dpg

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if a.calib_copy:
        n = 1 << 29   # 4 GiB of float64
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n * 8}))
        return

    ctx = dpg.Context(p_max=11)
    if a.condense_only:
        print(json.dumps({"condense_h1_p7": run_condense(ctx, dpg, stream)}), flush=True)
        ctx.close()
        return
    if a.aniso_only:
        print(json.dumps({"aniso_orders": run_aniso(ctx, dpg, stream)}), flush=True)
        ctx.close()
        return
    E, space, p = 4096, "H1", 7
    X = torch.from_numpy(meshgen.perturbed_hexes(E, noise=0.15, seed=1712)).cuda()
    m = dpg.packed_len(space, p)
    dt = torch.float64 if a.prec == "fp64" else torch.float32
    out = torch.empty(E * m, dtype=dt, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] workload: {E} x {space} p={p} {a.prec}, output {out.numel() * out.element_size() / 1e9:.2f} GB")

    # autotune the work decomposition on this workload (outside the timed region)
    slab_group = ctx.autotune(space, p, X, out=out, prec=a.prec, stream=stream)
    log(f"[bench] autotuned slab group: {slab_group}")

    def step():
        ctx.gram(space, p, X, out=out, prec=a.prec, stream=stream)

    wall, per = time_launches(step, a.steps, a.warmup, stream)
    ms_per_step = 1e3 * wall / a.steps
    value = E * a.steps / wall
    kern_ms = float(np.mean(per))
    flops = dpg.general_flops(space, p) * E              # stage xi2 over every (i2, j2) of each pair
    flops_trim = dpg.general_flops_trimmed(space, p) * E  # diagonal pairs' stage xi2 over i2 <= j2 only
    out_bytes = m * out.element_size() * E
    alg_bytes = out_bytes + 24 * 8 * E
    peak = PEAK_FP64_TFLOPS if a.prec == "fp64" else PEAK_FP32_TFLOPS
    achieved = flops / (kern_ms * 1e-3) / 1e12
    traffic = measured_traffic("bytes_per_launch_" + a.prec)
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel": f"k_general<H1,p=7,{'double' if a.prec == 'fp64' else 'float'}>",
            "avg_launch_ms": round(kern_ms, 4),
            "algorithmic": {"flops_per_launch": flops, "bytes_per_launch": alg_bytes,
                            "flops_per_launch_trimmed": flops_trim,
                            "tflops_trimmed": round(flops_trim / (kern_ms * 1e-3) / 1e12, 3),
                            "hbm_gbs_achieved": round(alg_bytes / (kern_ms * 1e-3) / 1e9, 1),
                            "hbm_frac": round(alg_bytes / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}}
    log(f"[bench] {value:.4g} elem/s, kernel {kern_ms:.3f} ms, {achieved:.2f} TFLOP/s, "
        f"{alg_bytes / (kern_ms * 1e-3) / 1e9:.0f} GB/s")

    # correctness spot check of the timed output (one element against the oracle is done in tests;
    # here only cheap invariants: finite, positive diagonal)
    d = torch.arange(dpg.gram_dim(space, p), device="cuda")
    diag = out.view(E, m)[:, d * (d + 1) // 2 + d]
    assert bool(torch.isfinite(diag).all()) and bool((diag > 0).all())

    extra = {}
    if a.extra:
        extra = run_extra(ctx, dpg, stream, E, X, out)
    del out
    torch.cuda.empty_cache()
    if a.extra:
        extra["batched_mixed_50000"] = run_mixed_full(ctx, dpg, stream)
        extra["orders_p4_p10"] = run_orders(ctx, dpg, stream)
        extra["scaling"] = run_scaling(ctx, dpg, stream)
        extra["latency"] = run_latency(ctx, dpg, stream)
    serving = None
    if a.serve_seconds > 0:
        serving = run_serving(ctx, dpg, a.serve_seconds)

    cpu = None
    if not a.no_cpu:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline()

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "elements/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.prec == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": "4096 trilinear hexes (unit cube vertices + U(-0.15,0.15) noise, seed 1712), "
                               "H1 test Gram p+dp=7, 8^3 Gauss-Legendre points, general O(p^7) path, packed output",
                   "n_elem": E, "space": space, "p": p, "points_per_dir": 8,
                   "output_bytes": out_bytes, "slab_group": slab_group},
        "roofline": roof, "cpu_baseline": cpu, "serving": serving, "extra": extra,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def run_condense(ctx, dpg, stream):
    import numpy as np
    import torch

    import meshgen

    # static condensation on the device: Cholesky factor of the benchmark's Grams in place, then
    # G^{-1} B for 343 right-hand sides (the H1 trial space of order 6 of the Poisson example)
    n_c, sp_c, p_c, nrhs_c = 1024, "H1", 7, 343
    nn = dpg.gram_dim(sp_c, p_c)
    mc = nn * (nn + 1) // 2
    Xc = torch.from_numpy(meshgen.perturbed_hexes(n_c, noise=0.15, seed=1713)).cuda()
    gsrc = ctx.gram(sp_c, p_c, Xc, stream=stream)
    work = torch.empty_like(gsrc)
    info = torch.empty(n_c, dtype=torch.int32, device="cuda")
    fr = []
    for it in range(6):
        work.copy_(gsrc)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.cholesky(work, nn, info=info, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if it:
            fr.append(e0.elapsed_time(e1))
    assert int(info.abs().sum()) == 0, "benchmark Grams must factor"
    kf = float(np.mean(fr))
    flops_f = n_c * (nn ** 3 / 3.0 + nn ** 2 / 2.0)
    bmat = torch.randn(n_c, nrhs_c, nn, dtype=torch.float64, device="cuda")
    w, pr = time_launches(lambda: ctx.cholesky_solve(work, nn, bmat, stream=stream), 3, 1, stream)
    ks = float(np.mean(pr))
    flops_s = n_c * 2.0 * nn * nn * nrhs_c
    row = {
        "n_elem": n_c, "n": nn, "nrhs": nrhs_c,
        "cholesky_ms": round(kf, 3), "cholesky_tflops": round(flops_f / (kf * 1e-3) / 1e12, 2),
        "cholesky_frac_fp64": round(flops_f / (kf * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
        "solve_ms": round(ks, 3), "solve_tflops": round(flops_s / (ks * 1e-3) / 1e12, 2),
        "solve_frac_fp64": round(flops_s / (ks * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
    log(f"[bench] extra condense {row}")
    del gsrc, work, bmat, Xc
    torch.cuda.empty_cache()
    return row


def run_aniso(ctx, dpg, stream):
    """Non-uniform orders (p1, p2, p3), one rule per coordinate: the route the entry point
    takes (orders embedded in the uniform kernel of order max p_d; equal orders the uniform
    kernel itself) and the per-direction kernel (least order outermost)."""
    import numpy as np
    import torch
    import meshgen
    ani = []
    for space, q in (("H1", (7, 6, 5)), ("H1", (7, 7, 7)), ("HCURL", (6, 5, 4)), ("HDIV", (5, 6, 4)),
                     ("L2", (8, 7, 6))):
        nd = dpg.gram_dim_aniso(space, q)
        mm = nd * (nd + 1) // 2
        n_a = int(min(4096, (2 << 30) // (mm * 8)))
        Xa = torch.from_numpy(meshgen.perturbed_hexes(n_a, noise=0.15, seed=1712)).cuda()
        o = torch.empty(n_a * mm, dtype=torch.float64, device="cuda")
        w, pr = time_launches(lambda: ctx.gram_aniso(space, q, Xa, out=o, stream=stream), 3, 1, stream)
        kk = float(np.mean(pr))
        route = ctx.aniso_route(space, q)
        row = {"space": space, "p": list(q), "n_elem": n_a, "route": route, "kernel_ms": round(kk, 3),
               "elements_per_s": round(n_a / (kk * 1e-3), 1),
               "hbm_gbs": round(mm * 8 * n_a / (kk * 1e-3) / 1e9, 1)}
        w, pr = time_launches(lambda: ctx.gram_aniso(space, q, Xa, out=o, path="general", stream=stream),
                              3, 1, stream)
        row["per_direction_ms"] = round(float(np.mean(pr)), 3)
        ani.append(row)
        log(f"[bench] extra aniso {row}")
        del o, Xa
        torch.cuda.empty_cache()
    return ani


def run_extra(ctx, dpg, stream, E, X, out64):
    """FP32 on the benchmark workload; affine and extruded reduced vs general;
    an uneven-order batch.  Small repeat counts; every rate is elements/s."""
    import numpy as np
    import torch

    import meshgen
    res = {}
    m = dpg.packed_len("H1", 7)
    out32 = torch.empty(E * m, dtype=torch.float32, device="cuda")
    ctx.autotune("H1", 7, X, out=out32, prec="fp32", stream=stream)
    wall, per = time_launches(lambda: ctx.gram("H1", 7, X, out=out32, prec="fp32", stream=stream), 10, 2, stream)
    k = float(np.mean(per))
    fl = dpg.general_flops("H1", 7) * E
    res["h1_p7_fp32"] = {"elements_per_s": round(E * 10 / wall, 1), "kernel_ms": round(k, 4),
                         "tflops": round(fl / (k * 1e-3) / 1e12, 2),
                         "frac_fp32_mfma_peak": round(fl / (k * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
                         "hbm_gbs": round((m * 4 + 192) * E / (k * 1e-3) / 1e9, 1)}
    del out32
    torch.cuda.empty_cache()
    log(f"[bench] extra fp32: {res['h1_p7_fp32']}")

    res["affine_reduced_vs_general"] = run_config3(ctx, dpg, stream)

    # extruded elements (quadrilaterals extruded along x1): reduced (exact xi1 integrals) vs general
    ext = []
    for space, p in (("H1", 4), ("H1", 7), ("HCURL", 6), ("HDIV", 6), ("L2", 8)):
        mm = dpg.packed_len(space, p)
        n_e = int(min(4096, (4 << 30) // (mm * 8)))
        X_e = torch.from_numpy(meshgen.extruded_prisms(n_e, seed=1716)).cuda()
        o = torch.empty(n_e * mm, dtype=torch.float64, device="cuda")
        row = {"space": space, "p": p, "n_elem": n_e}
        for path in ("reduced", "general"):
            ctx.autotune(space, p, X_e, kind="extruded", out=o, path=path, stream=stream)
            w, pr = time_launches(lambda: ctx.gram(space, p, X_e, kind="extruded", out=o, path=path,
                                                   stream=stream), 5, 1, stream)
            kk = float(np.mean(pr))
            row[path] = {"elements_per_s": round(n_e * 5 / w, 1), "kernel_ms": round(kk, 4),
                         "hbm_gbs": round((mm * 8 + 80) * n_e / (kk * 1e-3) / 1e9, 1),
                         "hbm_frac": round((mm * 8 + 80) * n_e / (kk * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        ext.append(row)
        log(f"[bench] extra extruded {row}")
        del o, X_e
        torch.cuda.empty_cache()
    res["extruded_reduced_vs_general"] = ext

    # vector-valued test spaces: block-diagonal replication of packed Grams (copies = 3), HBM-bound copy
    n_r, sp_r, p_r = 1024, "H1", 7
    nn = dpg.gram_dim(sp_r, p_r)
    src = torch.ones(n_r * (nn * (nn + 1) // 2), dtype=torch.float64, device="cuda")
    dst = torch.empty(n_r * (3 * nn * (3 * nn + 1) // 2), dtype=torch.float64, device="cuda")
    w, pr = time_launches(lambda: ctx.replicate_blocks(src, nn, 3, out=dst, stream=stream), 5, 1, stream)
    kk = float(np.mean(pr))
    moved = (src.numel() + dst.numel()) * 8
    res["replicate_h1_p7_x3"] = {"n_elem": n_r, "kernel_ms": round(kk, 4), "gb_moved": round(moved / 1e9, 2),
                                 "hbm_gbs": round(moved / (kk * 1e-3) / 1e9, 1),
                                 "hbm_frac": round(moved / (kk * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    log(f"[bench] extra replicate {res['replicate_h1_p7_x3']}")
    del src, dst
    res["aniso_orders"] = run_aniso(ctx, dpg, stream)

    res["condense_h1_p7"] = run_condense(ctx, dpg, stream)
    # adjoint graph coupling block (one constant matrix per order)
    cpl = ctx.adjoint_coupling(11)
    w, pr = time_launches(lambda: ctx.adjoint_coupling(11, out=cpl, stream=stream), 5, 1, stream)
    res["adjoint_coupling_p11"] = {"shape": list(cpl.shape), "kernel_ms": round(float(np.mean(pr)), 4)}
    del cpl
    torch.cuda.empty_cache()

    # uneven batch, scaled-down version of the 50,000-element mixed run
    n_b = 8000
    sp, pr_, G = meshgen.mixed_batch(n_b, p_lo=2, p_hi=9, dp=1, seed=1714)
    lens = np.array([dpg.packed_len(int(s), int(q)) for s, q in zip(sp, pr_)], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    ob = torch.empty(int(lens.sum()), dtype=torch.float64, device="cuda")
    args = (torch.from_numpy(sp).cuda(), torch.from_numpy(pr_).cuda(), torch.from_numpy(G).cuda(),
            torch.from_numpy(off).cuda(), ob)
    w, pr = time_launches(lambda: ctx.gram_batched(*args, stream=stream), 3, 1, stream)
    res["batched_mixed_8000_fp64"] = {"elements_per_s": round(n_b * 3 / w, 1), "ms_per_call": round(1e3 * w / 3, 3),
                                      "output_gb": round(float(lens.sum()) * 8 / 1e9, 2),
                                      "hbm_gbs": round(float(lens.sum()) * 8 / (w / 3) / 1e9, 1)}
    log(f"[bench] extra batched {res['batched_mixed_8000_fp64']}")
    del ob
    torch.cuda.empty_cache()
    return res


def run_config3(ctx, dpg, stream, n_elem=20000, chunk_bytes=48 << 30, n_check=6):
    """20,000 affine parallelepipeds (J = (I + S) diag(lam), seed 1713), H(curl) and
    H(div) at p = 4, 6, 8: the reduced O(p^6) path and the general O(p^7) path at the
    full element count.  Outputs above chunk_bytes (p = 8: 302 / 239 GB) run as
    consecutive element chunks through two reused buffers; before a chunk's buffers
    are reused, n_check of its elements are compared between the two paths
    (max |reduced - general| <= 1e-12 max |reduced|; both are pinned to the oracle by
    the tests).  Kernel times are event-timed per chunk and summed."""
    import numpy as np
    import torch

    import meshgen
    A_all = meshgen.affine_parallelepipeds(n_elem, seed=1713)
    rows = []
    for space in ("HCURL", "HDIV"):
        for p in (4, 6, 8):
            mm = dpg.packed_len(space, p)
            per = max(1, min(n_elem, chunk_bytes // (mm * 8)))
            bufs = {k: torch.empty(per * mm, dtype=torch.float64, device="cuda") for k in ("reduced", "general")}
            ms = {"reduced": 0.0, "general": 0.0}
            worst = 0.0
            chunks = 0
            rng = np.random.default_rng(p)
            for c0 in range(0, n_elem, per):
                c1 = min(n_elem, c0 + per)
                A = torch.from_numpy(np.ascontiguousarray(A_all[c0:c1])).cuda()
                for path in ("reduced", "general"):
                    ctx.gram(space, p, A, kind="affine", out=bufs[path], path=path, stream=stream)   # warm
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    ctx.gram(space, p, A, kind="affine", out=bufs[path], path=path, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ms[path] += e0.elapsed_time(e1)
                for e in rng.integers(0, c1 - c0, n_check):
                    r = bufs["reduced"][e * mm:(e + 1) * mm]
                    g = bufs["general"][e * mm:(e + 1) * mm]
                    worst = max(worst, float((r - g).abs().max() / r.abs().max()))
                chunks += 1
                del A
            assert worst <= 1e-12, f"config 3 {space} p={p}: reduced vs general {worst:.3e}"
            out_b = float(mm * 8 + 96) * n_elem
            row = {"space": space, "p": p, "n_elem": n_elem, "chunks": chunks, "output_gb": round(out_b / 1e9, 1),
                   "sample_max_rel_diff": worst}
            for path in ("reduced", "general"):
                row[path] = {"kernel_ms": round(ms[path], 3), "elements_per_s": round(n_elem / (ms[path] * 1e-3), 1),
                             "hbm_gbs": round(out_b / (ms[path] * 1e-3) / 1e9, 1),
                             "hbm_frac": round(out_b / (ms[path] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
            rows.append(row)
            log(f"[bench] config 3 {row}")
            del bufs
            torch.cuda.empty_cache()
    return rows


# The paper's own single-element timings (seconds per element; one element equal to the
# master hexahedron; hardware, compiler and precision not stated), context only:
# Table 1 (H1 Gram of the Poisson primal test space) and Table 3 (H(curl) Gram of the
# Maxwell primal test space), tensorization and simplified tensorization columns.
PAPER_SECONDS = {
    ("H1", "tensorization"): {2: 1.64e-3, 3: 1.95e-3, 4: 3.31e-3, 5: 6.70e-3, 6: 1.49e-2, 7: 3.05e-2},
    ("H1", "simplified"): {2: 1.67e-3, 3: 1.89e-3, 4: 2.85e-3, 5: 4.96e-3, 6: 9.45e-3, 7: 1.80e-2},
    ("HCURL", "tensorization"): {2: 3.41e-2, 3: 3.98e-2, 4: 5.39e-2, 5: 9.42e-2, 6: 0.203, 7: 0.464},
    ("HCURL", "simplified"): {2: 3.17e-2, 3: 3.32e-2, 4: 3.67e-2, 5: 5.02e-2, 6: 7.88e-2, 7: 0.132},
}


def run_latency(ctx, dpg, stream, reps=200):
    """Single-element calls: config 1 (the cube (0,2)^3, H1, p = 3) and one element
    equal to the master hexahedron (the paper's timing workload) for H1 and H(curl) at
    p = 2..7, on the general path (trilinear input) and the reduced path (affine
    identity).  Per call: the kernel time (events) and the host-side latency of the
    call plus a stream synchronisation (median over reps), beside the paper's seconds
    per element (Tables 1 and 3, hardware unstated) as context."""
    import numpy as np
    import torch

    import meshgen

    def timed(fn):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        k, h = [], []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            h.append(time.perf_counter() - t0)
            k.append(e0.elapsed_time(e1))
        return round(float(np.median(k)) * 1e3, 2), round(float(np.median(h)) * 1e6, 1)

    out = {}
    cube = torch.from_numpy(meshgen.scaled_cube(2.0)).cuda()
    o = ctx.gram("H1", 3, cube)
    k, h = timed(lambda: ctx.gram("H1", 3, cube, out=o, stream=stream))
    out["config1_h1_p3_cube"] = {"kernel_us": k, "call_us_p50": h}
    log(f"[bench] config 1 latency: kernel {k} us, call + sync {h} us")
    unit = torch.from_numpy(meshgen.scaled_cube(1.0)).cuda()
    ident = torch.zeros(12, dtype=torch.float64, device="cuda")
    ident[3:] = torch.eye(3, dtype=torch.float64, device="cuda").reshape(-1)
    rows = []
    for space in ("H1", "HCURL"):
        for p in range(2, 8):
            o = ctx.gram(space, p, unit)
            kg, hg = timed(lambda: ctx.gram(space, p, unit, out=o, stream=stream))
            kr, hr = timed(lambda: ctx.gram(space, p, ident, kind="affine", out=o, stream=stream))
            rows.append({"space": space, "p": p, "general_kernel_us": kg, "general_call_us": hg,
                         "reduced_kernel_us": kr, "reduced_call_us": hr,
                         "paper_tensorization_s": PAPER_SECONDS[(space, "tensorization")][p],
                         "paper_simplified_s": PAPER_SECONDS[(space, "simplified")][p]})
    out["identity_element"] = rows
    out["paper_hardware"] = "not stated in the paper"
    log(f"[bench] identity element rows: {rows}")
    return out


def run_orders(ctx, dpg, stream, out_bytes=2 << 30):
    """The metric's per-order figures: every space at p = 4..10 on the general
    (quadrature) path, FP64, perturbed hexes (seed 7), about out_bytes of output per
    launch (at most 8192 elements), the shipped tuning table's schedules.  Each row:
    elements/s and the fraction of its roofline 1 / max(F / 78.6 TFLOP/s,
    B / 8 TB/s) per element, F = the staged contraction's algorithmic flops, B = the
    packed output + 192 B of trilinear geometry."""
    import numpy as np
    import torch

    import meshgen
    rows = []
    for space in ("H1", "HCURL", "HDIV", "L2"):
        for p in range(4, 11):
            m = dpg.packed_len(space, p)
            n = int(max(16, min(8192, out_bytes // (m * 8))))
            g = torch.from_numpy(meshgen.perturbed_hexes(n, seed=7)).cuda()
            o = torch.empty(n * m, dtype=torch.float64, device="cuda")
            w, per = time_launches(lambda: ctx.gram(space, p, g, out=o, stream=stream), 5, 3, stream)
            ms = float(np.mean(per))
            F = dpg.general_flops(space, p)
            B = m * 8 + 192
            t_roof = max(F / (PEAK_FP64_TFLOPS * 1e12), B / (PEAK_HBM_GBS * 1e9))
            eps = n / (ms * 1e-3)
            rows.append({"space": space, "p": p, "n_elem": n, "kernel_ms": round(ms, 4), "elements_per_s": round(eps, 1),
                         "roofline_elements_per_s": round(1 / t_roof, 1), "frac": round(eps * t_roof, 4),
                         "bound": "mfma" if F / (PEAK_FP64_TFLOPS * 1e12) > B / (PEAK_HBM_GBS * 1e9) else "hbm",
                         "tflops": round(F * eps / 1e12, 2), "hbm_gbs": round(B * eps / 1e9, 1)})
            del o, g
        torch.cuda.empty_cache()
    log(f"[bench] per-order fractions: {[(r['space'], r['p'], r['frac']) for r in rows]}")
    return rows


def run_scaling(ctx, dpg, stream, out_bytes=2 << 30):
    """Time per element against the order: the general path on perturbed hexes
    (H1) and the reduced path on affine elements (H(curl)), p = 2..11, FP64,
    with about out_bytes of output per launch (at most 4096 elements).  The
    slopes of log(time/element) over log p, fitted on p >= 6, are set beside
    the algorithmic exponents: flops ~ p^7 (general), output ~ p^6 (both)."""
    import numpy as np
    import torch

    import meshgen
    rows = {"general_H1": [], "reduced_HCURL": []}
    for key, space, kind in (("general_H1", "H1", "trilinear"), ("reduced_HCURL", "HCURL", "affine")):
        for p in range(2, 12):
            m = dpg.packed_len(space, p)
            n = int(max(16, min(4096, out_bytes // (m * 8))))
            if kind == "trilinear":
                g = torch.from_numpy(meshgen.perturbed_hexes(n, seed=7)).cuda()
            else:
                g = torch.from_numpy(meshgen.affine_parallelepipeds(n, seed=7)).cuda()
            o = torch.empty(n * m, dtype=torch.float64, device="cuda")
            w, per = time_launches(lambda: ctx.gram(space, p, g, kind=kind, out=o, stream=stream), 5, 2, stream)
            us = float(np.mean(per)) * 1e3 / n
            rows[key].append({"p": p, "n_elem": n, "us_per_elem": round(us, 4),
                              "mflop_per_elem": round(dpg.general_flops(space, p) / 1e6, 3),
                              "mb_per_elem": round(m * 8 / 1e6, 4)})
            del o, g
        torch.cuda.empty_cache()
    fit = {}
    for key, r in rows.items():
        sel = [x for x in r if x["p"] >= 6]
        lp = np.log([x["p"] for x in sel])
        fit[key] = {"time_exponent": round(float(np.polyfit(lp, np.log([x["us_per_elem"] for x in sel]), 1)[0]), 2),
                    "output_exponent": round(float(np.polyfit(lp, np.log([x["mb_per_elem"] for x in sel]), 1)[0]), 2)}
        if key.startswith("general"):
            fit[key]["flop_exponent"] = round(float(np.polyfit(lp, np.log([x["mflop_per_elem"] for x in sel]), 1)[0]), 2)
    log(f"[bench] scaling fit (p >= 6): {fit}")
    return {"rows": rows, "fit_p_ge_6": fit}


def run_mixed_full(ctx, dpg, stream, n_elem=50000, chunk_bytes=48 << 30):
    """The uneven-order batch at full size: 50,000 trilinear hexes, space
    uniform over the four, p uniform in 2..9 plus dp = 1 (seed 1714).  Its FP64
    output (~0.3 TB) exceeds device memory, so it runs as consecutive element
    chunks of at most chunk_bytes output, each one batched call into one
    reused buffer; the rate covers every chunk (planning included)."""
    import numpy as np
    import torch

    import meshgen
    sp, pr_, G = meshgen.mixed_batch(n_elem, p_lo=2, p_hi=9, dp=1, seed=1714)
    lens = np.array([dpg.packed_len(int(s), int(q)) for s, q in zip(sp, pr_)], dtype=np.int64)
    res = {"n_elem": n_elem, "output_gb_fp64": round(float(lens.sum()) * 8 / 1e9, 1)}
    for prec, es in (("fp64", 8), ("fp32", 4)):
        cuts, acc, start = [], 0, 0
        for e in range(n_elem):
            if acc + lens[e] * es > chunk_bytes and e > start:
                cuts.append((start, e))
                start, acc = e, 0
            acc += lens[e] * es
        cuts.append((start, n_elem))
        chunks = []
        for a0, a1 in cuts:
            off = np.concatenate([[0], np.cumsum(lens[a0:a1])[:-1]]).astype(np.int64)
            chunks.append((torch.from_numpy(sp[a0:a1].copy()).cuda(), torch.from_numpy(pr_[a0:a1].copy()).cuda(),
                           torch.from_numpy(np.ascontiguousarray(G[a0:a1])).cuda(), torch.from_numpy(off).cuda(),
                           int(lens[a0:a1].sum())))
        host = [(np.ascontiguousarray(sp[a0:a1]), np.ascontiguousarray(pr_[a0:a1])) for a0, a1 in cuts]
        buf = torch.empty(max(c[4] for c in chunks), dtype=torch.float64 if es == 8 else torch.float32,
                          device="cuda")

        def one_pass():
            # space/p from the host copies: a replayed plan is enqueued without reading them back
            for (s_, p_, g_, o_, _), (hs, hp) in zip(chunks, host):
                ctx.gram_batched_host(hs, hp, g_, o_, buf, prec=prec, stream=stream)

        one_pass()                      # plans (graph capture) and warm-up
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            one_pass()
        torch.cuda.synchronize()
        w = (time.perf_counter() - t0) / reps
        res[prec] = {"elements_per_s": round(n_elem / w, 1), "s_per_pass": round(w, 4), "chunks": len(chunks),
                     "hbm_gbs": round(float(lens.sum()) * es / w / 1e9, 1)}
        log(f"[bench] mixed 50000 {prec}: {res[prec]}")
        del buf, chunks
        torch.cuda.empty_cache()
    return res


def run_serving(ctx, dpg, seconds, warmup=5.0, rate_hz=200.0, seed=1715, chunk_bytes=8 << 30):
    """Replay a Poisson serving trace through the serving loop (dpg_serve_*).

    Requests: 64..2048 trilinear hexes, space uniform, p uniform in 2..10 plus
    dp = 1, FP64, arriving at rate_hz for warmup + seconds.  The client submits
    each request at its arrival time with dpg_serve_submit_chunked: the server
    cuts it into element chunks of at most chunk_bytes output (a 2048-element
    H(curl) p = 11 request alone is 185 GB), polls, and releases each chunk as
    soon as it is complete.  Request latency = arrival -> last chunk pollable
    (server clock), over the requests arriving after the warm-up; the server's
    own statistics are per chunk and cover the whole trace."""
    import collections

    import numpy as np
    import torch

    import meshgen
    trace = meshgen.serving_trace(duration_s=warmup + seconds, rate_hz=rate_hz, n_lo=64, n_hi=2048, p_lo=2,
                                  p_hi=10, dp=1, seed=seed)
    geo = [meshgen.perturbed_hexes(r["n_elem"], seed=r["seed"]).reshape(-1) for r in trace]
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(192 << 30, free - (24 << 30)))
    srv = dpg.Server(ctx, mem_budget_bytes=budget, max_slots=1 << 21, max_inflight=256, max_queue=1 << 16,
                     n_streams=4, max_merge=32)
    # every (space, order) once, so code-object loading is not in the trace
    warm = [srv.submit(sp, q, meshgen.perturbed_hexes(64, seed=1).reshape(-1), dp=1)
            for sp in range(4) for q in range(2, 11)]
    pend = set(warm)
    while pend:
        for t in list(pend):
            if srv.poll(t) is not None:
                srv.release(t)
                pend.discard(t)
    srv.reset_stats()

    offered = 0.0
    backlog = collections.deque()           # requests not yet accepted (queue full)
    owner, left, t_done = {}, {}, {}
    arrival_srv, lag = {}, {}
    i = 0
    t0 = time.perf_counter()
    while i < len(trace) or backlog or owner:
        now = time.perf_counter() - t0
        while i < len(trace) and trace[i]["t"] <= now:
            backlog.append(i)
            i += 1
        while backlog:
            ri = backlog[0]
            r = trace[ri]
            try:
                first, k, _ = srv.submit_chunked(r["space"], r["p"], geo[ri], dp=r["dp"], max_chunk_bytes=chunk_bytes)
            except dpg.DpgError as e:
                if e.code == dpg.EAGAIN:
                    break
                raise
            backlog.popleft()
            lag[ri] = (time.perf_counter() - t0) - r["t"]      # how late the client submitted
            left[ri] = k
            for t in range(first, first + k):
                owner[t] = ri
            if r["t"] >= warmup:
                offered += r["n_elem"] * dpg.packed_len(r["space"], r["p"] + r["dp"]) * 8
        for t in list(owner):
            res = srv.poll(t)
            if res is None:
                continue
            ri = owner.pop(t)
            assert res["status"] == dpg.OK
            # arrival on the server clock: the chunk's t_submit minus the client's lag
            arrival_srv.setdefault(ri, res["t_submit"] - lag[ri])
            t_done[ri] = max(t_done.get(ri, 0.0), res["t_done"])
            left[ri] -= 1
            srv.release(t)
        if not backlog and i < len(trace):
            time.sleep(max(0.0, min(5e-4, trace[i]["t"] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    assert not any(left.values())
    st = srv.stats()
    meas = [k for k in range(len(trace)) if trace[k]["t"] >= warmup]
    lat = np.array([t_done[k] - arrival_srv[k] for k in meas])
    elems = sum(trace[k]["n_elem"] for k in meas)
    out_b = sum(trace[k]["n_elem"] * dpg.packed_len(trace[k]["space"], trace[k]["p"] + trace[k]["dp"]) * 8
                for k in meas)
    span = max(t_done[k] for k in meas) - min(arrival_srv[k] for k in meas)
    out = {
        "requests": len(meas), "warmup_requests": len(trace) - len(meas), "rate_hz": rate_hz,
        "duration_s": seconds, "warmup_s": warmup, "elements": elems,
        "elements_per_s": round(elems / span, 1), "output_tb_per_s": round(out_b / span / 1e12, 3),
        "offered_tb_per_s": round(offered / seconds / 1e12, 3),
        "latency_p50_ms": round(1e3 * float(np.percentile(lat, 50, method="inverted_cdf")), 3),
        "latency_p99_ms": round(1e3 * float(np.percentile(lat, 99, method="inverted_cdf")), 3),
        "latency_max_ms": round(1e3 * float(lat.max()), 3),
        "chunk_latency_p50_ms": round(1e3 * st["lat_p50"], 3), "chunk_latency_p99_ms": round(1e3 * st["lat_p99"], 3),
        "chunk_wait_p99_ms": round(1e3 * st["wait_p99"], 3),
        "chunks": st["completed"], "launches": st["launches"], "max_concurrent_launches": st["max_concurrent_launches"],
        "budget_gb": round(budget / 1e9, 1), "peak_admitted_gb": round(st["peak_admitted_bytes"] / 1e9, 1),
        "client_submit_lag_p99_ms": round(1e3 * float(np.percentile([lag[k] for k in meas], 99)), 3),
        "wall_s": round(wall, 2),
        "precision": "fp64", "chunk_gb": round(chunk_bytes / 1e9, 1), "chunking": "server (dpg_serve_submit_chunked)",
    }
    log(f"[bench] serving: {out}")
    srv.close()
    return out


if __name__ == "__main__":
    main()
