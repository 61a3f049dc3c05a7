"""Approximate selected inversion from an incomplete LDL^T on AMD MI355X.

The compute path is libasi.so (HIP kernels for gfx950 behind the C ABI in
include/asi.h); ``asi`` is its thin ctypes binding.
"""
from .asi import AsiError, Solver, dense_symeig, load_library, upload_factors  # noqa: F401
