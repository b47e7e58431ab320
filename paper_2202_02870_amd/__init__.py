"""MI355X-native *_L-product tensor completion.

The compute path is the HIP library `liblt.so` (C-ABI, declared in
include/lt.h); `paper_2202_02870_amd.lt` is its thin ctypes binding.  Importing
this package does not load the library; `paper_2202_02870_amd.lt` does, and
raises if it is missing.
"""
__all__ = ["workloads"]
