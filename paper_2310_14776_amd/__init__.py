"""MI355X (gfx950) library for one block step of the real-space FD-PAW
eigensolver: H~psi, S~psi, projector overlaps, subspace matrices, FP64
generalised eigensolve and rotation, behind the C ABI in include/gpaw_fd.h.
A precision form (single-precision storage, split-BF16 matrix-core
products) and a batched form (many systems in one graph launch) use the same
calls. Beside the step: density and atomic density matrices, the Davidson
update, and a zero-boundary multigrid Poisson solver with its grid
transfers.
"""
from ._binding import (System, Batch, GpawError, load, library_path, ENTRY_POINTS,
                       GPAW_F64, GPAW_C128, GPAW_F32, GPAW_C64, probe_copy, probe_mfma,
                       Poisson, laplacian_zero, grid_restrict, grid_interpolate)

__all__ = ["System", "Batch", "GpawError", "load", "library_path", "ENTRY_POINTS",
           "GPAW_F64", "GPAW_C128", "GPAW_F32", "GPAW_C64", "probe_copy", "probe_mfma",
           "Poisson", "laplacian_zero", "grid_restrict", "grid_interpolate"]
