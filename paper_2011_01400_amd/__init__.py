"""MI355X-native imaginary-frequency LRI-G0W0 screening and self-energy.

The compute lives in liblrigw.so (HIP, gfx950; interface in include/lrigw.h).
`paper_2011_01400_amd.lrigw` is its ctypes binding.
"""
__all__ = ["lrigw", "build"]
