"""MI355X-native weighted k-means++ seeding and Lloyd iterations.

The computation lives in libkmx.so (HIP kernels for gfx950 behind the C ABI
of include/kmx.h); ``paper_1502_04265_amd.kmx`` is its ctypes binding.
"""
from . import kmx  # noqa: F401

__all__ = ["kmx"]
