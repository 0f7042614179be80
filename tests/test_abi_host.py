"""CPU checks of the C-ABI library (no GPU needed).

* every function declared in include/dpg.h is exported by libdpg.so;
* host-side helpers: dimensions, packed lengths, flop counts;
* the library's own tables (Gauss-Legendre by Newton iteration, chi/chi' by
  recursion, the closed-form F chart) equal the oracle's independently
  computed ones.
"""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import closed_forms, poly1d, quadrature, shapes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpg.h")


@pytest.fixture(scope="module")
def dpg():
    from tests._lib import load_binding
    return load_binding()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpg_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported(dpg):
    out = subprocess.run(["nm", "-D", "--defined-only", dpg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (dpg_[a-z0-9_]+)$", out, flags=re.M))
    decl = declared_functions()
    assert decl, "no declarations parsed"
    missing = [d for d in decl if d not in exported]
    assert not missing, missing
    for d in decl:
        assert hasattr(dpg._lib, d)


SP = {"H1": 0, "HCURL": 1, "HDIV": 2, "L2": 3}


def test_dimensions(dpg):
    for name, sid in SP.items():
        for p in range(1, 12):
            n = shapes.dimension(name, p)
            assert dpg.gram_dim(sid, p) == n
            assert dpg.packed_len(sid, p) == n * (n + 1) // 2
        assert dpg.gram_dim(sid, 0) == -1 and dpg.gram_dim(sid, 12) == -1
    assert dpg.gram_dim(4, 3) == -1


# Algorithmic MFLOP per element of the staged contraction, p = 4..8 (stage xi2 over every
# (i2, j2) of each needed (i3, j3) pair), as tabulated for the benchmark configurations.
CONTRACT_MFLOP = {
    "H1": [0.52, 1.71, 4.71, 11.43, 25.13],
    "HCURL": [1.90, 6.79, 19.98, 50.95, 116.38],
    "HDIV": [0.65, 2.53, 7.88, 20.98, 49.60],
    "L2": [0.02, 0.10, 0.34, 0.98, 2.43],
}


def test_general_flops_table(dpg):
    for sp, vals in CONTRACT_MFLOP.items():
        for p, v in zip(range(4, 9), vals):
            assert abs(dpg.general_flops(sp, p) / 1e6 - v) <= 0.005 + 1e-9, (sp, p)


def test_general_flops_trimmed(dpg):
    """The trimmed count drops exactly the xi2 stage of the diagonal pairs below the
    (i2, j2) diagonal: 2 L^2 per merged term, l and (i2 > j2), R3 pairs per diagonal
    block; H1 has 9 merged terms (q slots), p + 1 functions and L = p + 1 points."""
    for p in range(1, 12):
        R = L = p + 1
        drop = R * (R * (R - 1) // 2) * 2 * L * L * 9
        assert dpg.general_flops("H1", p) - dpg.general_flops_trimmed("H1", p) == drop
    for sp in ("HCURL", "HDIV", "L2"):
        for p in range(1, 12):
            assert 0 < dpg.general_flops_trimmed(sp, p) <= dpg.general_flops(sp, p)
    assert dpg.general_flops("H1", 12) == -1 and dpg.general_flops_trimmed(7, 3) == -1
    # grows like p^7: ratio p=8 / p=7 ~ (9/8)^7
    r = dpg.general_flops("H1", 8) / dpg.general_flops("H1", 7)
    assert 1.8 < r < 2.6


@pytest.mark.parametrize("L", range(1, 13))
def test_library_tables_match_oracle(dpg, L):
    kmax = 12
    z, w, c, d = dpg.host_tables(L, kmax)
    zo, wo = quadrature.gauss_legendre_01(L)
    np.testing.assert_allclose(z, zo, rtol=0, atol=2e-16 * 4)
    np.testing.assert_allclose(w, wo, rtol=1e-14, atol=0)
    np.testing.assert_allclose(c, poly1d.chi(kmax, zo), rtol=0, atol=1e-14)
    np.testing.assert_allclose(d, poly1d.dchi(kmax, zo), rtol=0, atol=1e-14)


def test_library_ftables_match_oracle(dpg):
    kmax = 12
    for r in (0, 1):
        for s in (0, 1):
            F = dpg.host_ftable(r, s, kmax)
            ref = closed_forms.F_table(r, s, kmax).astype(np.float64)
            np.testing.assert_array_equal(F == 0, ref == 0)
            np.testing.assert_allclose(F, ref, rtol=5e-16, atol=0)   # a couple of ulp


def test_invalid_arguments(dpg):
    with pytest.raises(dpg.DpgError):
        dpg.host_tables(0, 3)
    with pytest.raises(dpg.DpgError):
        dpg.host_ftable(2, 0, 3)
