"""Plain FP64 CPU oracle of the FLAME Hall-MHD lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously correct reference that the
GPU library is checked against. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does, and it shares no code with
the HIP library (it imports nothing from the product package).

Modules, each following the paper passage named in its header:
  lattice      D3Q27 / D3Q7 constants (Sec. 3.1, 3.2, App. A)
  equilibrium  sixth-order Hermite f^(0), Maxwell-stress term, Hall magnetic equilibrium
  collision    central-moment collision: definition via T and its exact closed form
  current      J from the moments (3x3 system) or the curl stencil; div B estimate
  scheme       moments, collide, stream, initial state, node fields
  analytic     exact damped Hall-MHD wave (Sec. 4.1)
  diagnostics  FP64 reductions, shell spectra, dissipation spectra and energy transfer (Sec. 4.4)
  validation   dispersion, dissipation and viscosity error measures of the wave tests (Sec. 4.3)
  extended     the same step in extended precision, to expose the FP64 oracle's own rounding

Parity pins live in tests/test_oracle_*.py. Unpinned beyond invariants: the forcing
extension (momentum and field budgets are pinned; the scheme itself is not in the paper).
"""

from . import analytic, collision, current, diagnostics, equilibrium, lattice, scheme  # noqa: F401
from .scheme import Params, State, collide, fields, init_state, moments, rest_state, step, stream  # noqa: F401
