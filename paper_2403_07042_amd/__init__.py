"""MI355X-native solver of the quantum master equation for finite-dimensional
cavity-QED models (Jaynes-/Tavis-Cummings-Hubbard lattices).

The compute path is libqme.so: hand-written HIP kernels for gfx950 behind a
C ABI (include/qme.h).  This package is its thin Python binding.
"""
from . import _lib
from .api import (Batch, Solver, basis, evolve_with_selection, hamiltonian_coo,
                  propagator_increment, select_states)

__all__ = ["Batch", "Solver", "basis", "evolve_with_selection", "hamiltonian_coo",
           "propagator_increment", "select_states", "_lib"]
