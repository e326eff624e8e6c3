"""MI355X-native batched Fossen 6-DOF simulator (MarineGym's hot path).

The compute lives in libmg.so (HIP kernels for gfx950 behind the C ABI of
include/mg.h); :mod:`paper_2410_14117_amd.mg` is its Python binding.
"""
__all__ = ["mg"]
