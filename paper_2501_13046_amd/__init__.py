"""MI355X-native multigrid solve of the initial-data constraints (CTT form).

The compute path is libgrtmg.so (HIP kernels for gfx950 behind the C ABI in
include/grtmg.h); ``paper_2501_13046_amd.grtmg`` is its ctypes binding.
"""
__all__ = ["grtmg"]
