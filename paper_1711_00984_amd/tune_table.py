"""Write the tuning table shipped with the library (tune_gfx950.json).

    python -m paper_1711_00984_amd.tune_table [--out PATH] [--quick]

Runs dpg_autotune (slab groups per workgroup and, on the quadrature path, the
diagonal-pair schedule) for every space and order, in both precisions, on
seeded synthetic elements of each geometry kind at a few batch sizes, and
saves the winners with dpg_tune_save.  dpg_tables_build loads the table that
sits next to libdpg.so, so untuned callers (the batched and serving paths)
start from measured schedules.  Needs one gfx950 GPU; takes a few minutes.
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

DEFAULT_OUT = os.path.join(HERE, "tune_gfx950.json")
SIZES = (64, 512, 4096)            # batch sizes tuned (size classes 6, 9, 12)
MAX_OUT_BYTES = 6 << 30            # output cap per tuned case


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="one batch size, FP64 quadrature path only")
    a = ap.parse_args()

    import torch

    import meshgen
    from paper_1711_00984_amd import dpg

    torch.cuda.set_device(0)
    ctx = dpg.Context(p_max=dpg.P_MAX, tune_table=None)     # start from an empty table
    st = torch.cuda.current_stream()
    cases = [("trilinear", "general", prec) for prec in ("fp64", "fp32")]
    cases += [(kind, "reduced", prec) for kind in ("affine", "extruded") for prec in ("fp64", "fp32")]
    if a.quick:
        cases = cases[:1]
    sizes = SIZES[1:2] if a.quick else SIZES
    t0 = time.perf_counter()
    n_rows = 0
    for kind, path, prec in cases:
        es = 8 if prec == "fp64" else 4
        for space in ("H1", "HCURL", "HDIV", "L2"):
            for p in range(1, dpg.P_MAX + 1):
                m = dpg.packed_len(space, p)
                done = set()
                for n in sizes:
                    n = int(max(1, min(n, MAX_OUT_BYTES // (m * es))))
                    if n in done:
                        continue
                    done.add(n)
                    if kind == "trilinear":
                        g = meshgen.perturbed_hexes(n, seed=2000 + p)
                    elif kind == "affine":
                        g = meshgen.affine_parallelepipeds(n, seed=2000 + p)
                    else:
                        g = meshgen.extruded_prisms(n, seed=2000 + p)
                    g = torch.from_numpy(g).cuda()
                    out = torch.empty(n * m, dtype=torch.float64 if es == 8 else torch.float32, device="cuda")
                    best = ctx.autotune(space, p, g, kind=kind, out=out, prec=prec, path=path, stream=st)
                    n_rows += 1
                    print(f"[tune] {kind:9s} {path:7s} {prec} {space:5s} p={p:2d} n={n:5d}: {best} slabs/workgroup",
                          flush=True)
                    del out, g
                torch.cuda.empty_cache()
    ctx.tune_save(a.out)
    print(f"[tune] {n_rows} cases in {time.perf_counter() - t0:.0f} s -> {a.out}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
