"""MI355X-native Yee-FDTD stepper for gain-filled disordered inverted opals.

The compute path is the C-ABI library ``libfdtd.so`` (HIP kernels for gfx950)
declared in ``include/fdtd.h``; ``paper_0802_3775_amd.fdtd`` is its thin
ctypes binding.  Importing this package does not load the library.
"""
__all__ = ["workloads"]
