"""Build libdpg.so (HIP kernels for gfx950 + the C ABI) in the package directory.

    python -m paper_1711_00984_amd.build        # or: python paper_1711_00984_amd/build.py
    python -m paper_1711_00984_amd.build --incremental   # reuse up-to-date objects

Objects go to <repo>/_build/; the shared library to
paper_1711_00984_amd/libdpg.so, where the Python binding loads it.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdpg.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -packed-fp32-ops: no v_pk_{add,mul,fma}_f32 generation (host pass ignores it)
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include")]


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip") or f.endswith(".cpp"):
            out.append(os.path.join(CSRC, f))
    return out


def _deps_mtime(src):
    """Latest modification time of src and of every local header it includes, transitively
    (quoted includes resolved in csrc/ and include/)."""
    seen, todo, latest = set(), [src], 0.0
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(f):
            continue
        seen.add(f)
        latest = max(latest, os.path.getmtime(f))
        with open(f, errors="replace") as fh:
            for line in fh:
                line = line.strip()
                if line.startswith("#include") and '"' in line:
                    name = line.split('"')[1]
                    for d in (os.path.dirname(f), CSRC, os.path.join(ROOT, "include")):
                        cand = os.path.normpath(os.path.join(d, name))
                        if os.path.exists(cand):
                            todo.append(cand)
                            break
    return latest


def _compile(src, incremental=False):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _deps_mtime(src):
        return obj, 0.0, ""
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "is not a recognized feature for this target" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msgs}")
    return obj, time.time() - t0, msgs


def build(verbose=True, jobs=None, incremental=False):
    """Compile every source (incremental=True skips objects newer than their
    source and every header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt, msgs in ex.map(lambda f: _compile(f, incremental), srcs):
            objs.append(obj)
            if verbose and dt > 0:
                print(f"  compiled {os.path.basename(obj)} in {dt:.1f}s", flush=True)
                if msgs.strip():
                    print(msgs, flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"  linked {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
