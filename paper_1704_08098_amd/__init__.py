"""MI355X (gfx950) engine for the spatial public goods game sweep.

The hot path lives in libpgg.so (HIP kernels behind the C ABI of
include/pgg.h); ``pgg`` is its ctypes binding.  Importing the package loads
nothing: ``pgg.load()`` does, and raises if the library is not built.
"""
__all__ = ["pgg", "workloads"]
