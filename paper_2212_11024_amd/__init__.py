"""MI355X-native coupled Hall-MHD lattice-Boltzmann step (FLAME scheme, arXiv 2212.11024).

The computation lives in libflame.so (HIP, gfx950; C ABI in include/flame.h). ``_lib`` binds
its entry points under the same names; ``Solver`` owns the device buffers of one run.
"""

from . import _lib  # noqa: F401
from ._lib import FlameError, load  # noqa: F401


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
