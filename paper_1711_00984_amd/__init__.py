"""Sum-factorised DPG Gram-matrix integration on MI355X (gfx950).

The compute lives in libdpg.so (HIP kernels + C ABI, include/dpg.h); the
``dpg`` module is its ctypes binding.  Importing the binding fails loudly if
the library has not been built (``python -m paper_1711_00984_amd.build``).
"""
