"""MI355X-native damped, smoothing-regularised LSQR (pDSurfTomo's solver step).

The compute lives in liblsqr_mi355x.so (hand-written HIP for gfx950, C ABI
in include/lsqr_mi355x.h); this package is the build script and a ctypes
binding.
"""
from .lsqr import (CSR, Info, LsqrError, Solver, Trainer, assemble_polylines, assemble_rays,  # noqa: F401
                   header_functions, load, rays_size, solve_batched, solve_batched_refined,
                   split_polylines)

__all__ = ["Solver", "Trainer", "LsqrError", "load", "header_functions", "solve_batched",
           "solve_batched_refined",
           "assemble_rays", "assemble_polylines", "split_polylines", "rays_size"]
