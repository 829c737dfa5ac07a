"""Seeded synthetic inputs for the FD-PAW block eigensolver step.

This package holds random draws and the input fields built from them (atom
positions, the local potential, the PAW correction matrices and the starting
block of wave functions). It holds none of the method's arithmetic: the
stencil, the projector functions, the projections, the subspace matrices, the
eigensolve and the rotation live in the HIP library and, independently, in
the CPU oracle. Both sides read the same arrays from here.
"""
from .systems import (System, make_system, standard_channels, config_system,
                      CONFIGS, ragged_cases, batched_systems, noise_band, smooth_band)
from .device import block_to_device

__all__ = ["System", "make_system", "standard_channels", "config_system",
           "CONFIGS", "ragged_cases", "batched_systems", "noise_band", "smooth_band",
           "block_to_device"]
