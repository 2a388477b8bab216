"""MI355X-native high-order immersed-interface Poisson solver.

The product is the HIP library libiim.so (C ABI in include/iim.h); the
Python module ``paper_2503_22455_amd.iim`` is a thin ctypes binding over it.
Nothing is loaded at import time.
"""
__all__ = ["iim", "build"]
