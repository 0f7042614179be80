"""Host test of the launch splitting arithmetic (csrc/launch_limits.h): large
batches are cut into launches that each stay under the dispatch limits."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_launch_limits(tmp_path):
    exe = tmp_path / "launch_limits"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_1711_00984_amd", "csrc"),
                    os.path.join(ROOT, "tests", "launch_limits_driver.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
