"""MI355X-native many-beam RHEED/TRHEPD forward model and adjoint (arXiv 2306.00271).

The computation lives in ``librheed.so`` (HIP kernels for gfx950 behind the
C ABI of ``include/rheed.h``); ``api`` is a thin torch/ctypes binding.
Importing ``api`` loads the library and raises if it has not been built.
"""
__all__ = ["api", "build"]
