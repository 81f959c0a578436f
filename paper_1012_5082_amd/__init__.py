"""MI355X-native VC-SGC transmutation Monte Carlo and EAM molecular dynamics.

The compute path is the HIP library built from ``csrc/`` (``libvcsgc.so``),
reached through the C ABI declared in ``include/vcsgc.h``; ``binding`` wraps
it with ctypes.  Importing the package does not load the library.
"""
__all__ = ["inputs"]
