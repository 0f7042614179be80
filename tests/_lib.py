"""Test helper: load the ctypes binding, building libdpg.so first if it is absent."""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_binding():
    lib = os.path.join(ROOT, "paper_1711_00984_amd", "libdpg.so")
    if not os.path.exists(lib):
        from paper_1711_00984_amd import build
        build.build(verbose=False)
    from paper_1711_00984_amd import dpg
    return dpg
