"""MI355X-native damped, smoothing-regularised LSQR (pDSurfTomo's solver step).

The compute lives in liblsqr_mi355x.so (hand-written HIP for gfx950, C ABI
in include/lsqr_mi355x.h); this package is the build script and a ctypes
binding.
"""
from .lsqr import (CSR, Info, LsqrError, Solver, header_functions, load)  # noqa: F401

__all__ = ["Solver", "LsqrError", "load", "header_functions"]
