"""MI355X-native Bloch-Maxwell eigensolver (block preconditioned inverse iteration with
multigrid, null-space elimination and Rayleigh-quotient extrapolation across Bloch
parameters), after Boerm, Koehl and Talebi, arXiv 2304.00337.

The computation lives in libbloch.so (HIP kernels for gfx950 behind the C ABI of
include/bloch.h); this package is its Python binding.  PyTorch provides device memory
and the stream.
"""
from .api import Batch, Server, Solver, batch_solve, raster_sources, to_device_block, from_device_block  # noqa: F401
from .native import OPS, load  # noqa: F401

__all__ = ["Solver", "Server", "Batch", "batch_solve", "raster_sources", "to_device_block", "from_device_block", "OPS", "load"]
