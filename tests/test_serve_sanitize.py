"""Sanitizer builds of the serving scheduler (host code only, CPU).

Builds tests/serve_sanitize_driver.cpp with the scheduler core and its timing
stub under ThreadSanitizer, then under AddressSanitizer + UBSan, and runs the
multi-threaded stress driver.  No HIP code is compiled or loaded.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_00984_amd", "csrc")
SRCS = [os.path.join(ROOT, "tests", "serve_sanitize_driver.cpp"), os.path.join(CSRC, "serve_core.cpp"),
        os.path.join(CSRC, "errors.cpp")]


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, san):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "drv")
    cmd = [gxx, "-std=c++20", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer", "-pthread",
           "-I", os.path.join(ROOT, "include"), *SRCS, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
