"""Seeded synthetic inputs shared by the CPU oracle tests, the GPU tests and the benchmark.

Every field here is an explicit list of Fourier modes, so the same seed gives the same
continuous field at every grid size. The module holds none of the lattice-Boltzmann
arithmetic: it only draws random numbers, builds mode lists and samples them on a grid.
"""

from .fields import (ModeField, half_space_wavevectors, shell_field, wave_field,
                     xia_field, orszag_tang, scaled, evaluate, evaluate_numpy)

__all__ = ["ModeField", "half_space_wavevectors", "shell_field", "wave_field", "xia_field",
           "orszag_tang", "scaled", "evaluate", "evaluate_numpy"]
