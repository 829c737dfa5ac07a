"""MI355X (gfx950) library for one block step of the real-space FD-PAW
eigensolver: H~psi, S~psi, projector overlaps, subspace matrices, FP64
generalised eigensolve and rotation, behind the C ABI in include/gpaw_fd.h.
"""
from ._binding import (System, GpawError, load, library_path, ENTRY_POINTS,
                       GPAW_F64, GPAW_C128)

__all__ = ["System", "GpawError", "load", "library_path", "ENTRY_POINTS",
           "GPAW_F64", "GPAW_C128"]
