"""MI355X (gfx950) exhaustive k-order epistasis scanner.

The compute path is ``libepi.so`` (HIP kernels + C++ runtime, C ABI in
``include/epi.h``); :mod:`paper_2201_02460_amd.epi` is its thin ctypes
binding.  Importing this package loads nothing; the binding loads the library
on first use and raises if it is missing.
"""
__all__ = ["epi", "build"]
