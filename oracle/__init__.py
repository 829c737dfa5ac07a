"""FP64 CPU oracle for the FD-PAW block eigensolver step.

TEST INFRASTRUCTURE ONLY. Imported by tests/, by __graft_entry__.smoke() and
by the cpu_baseline leg of bench.py; nothing in the product library calls it.
It shares no code with the HIP path: plain NumPy/SciPy in float64/complex128,
written from the paper's statement of the operators (Sec. "Projector
augmented-wave method", Eq. (dh) and the overlap operator beside it), the
FD representation (Sec. "Wave-function representations") and the subspace
diagonalisation step of the SCF loop (Sec. "Solving the Kohn-Sham equation").

Readings where the paper is silent (stencil order, Bloch boundary, projector
shapes, quadrature) are listed in each module's header.

Parity status: every function here is pinned by tests/test_oracle_*.py
against closed forms, brute force and library routines, except the
synthetic projector/potential definitions themselves, which stand in for
PAW setup files the paper's method reads and are therefore pinned only by
their own normalisation and harmonic checks ("parity unpinned" against a
real PAW dataset).
"""
from .stencil import WEIGHTS, laplacian, kinetic, symbol_1d
from .projectors import (radial_norm, solid_harmonics, projector_values,
                         projector_matrix, projector_matrix_sparse)
from .paw import project, addback, apply_H, apply_S, block_diag_atoms
from .subspace import (subspace_matrices, hermiticity_defect, diagonalize,
                       rotate, orthonormalize)
from .step import Operators, fd_step
from .density import pseudo_density, atomic_density_matrices, paw_norm
from .davidson import kinetic_diagonal, precondition, davidson_step
from . import poisson, tddft

__all__ = ["WEIGHTS", "laplacian", "kinetic", "symbol_1d", "radial_norm",
           "solid_harmonics", "projector_values", "projector_matrix",
           "projector_matrix_sparse",
           "project", "addback", "apply_H", "apply_S", "block_diag_atoms",
           "subspace_matrices", "hermiticity_defect", "diagonalize", "rotate",
           "orthonormalize",
           "Operators", "fd_step", "pseudo_density", "atomic_density_matrices", "paw_norm",
           "kinetic_diagonal", "precondition", "davidson_step", "poisson", "tddft"]
