"""Lattice constants of the two coupled schemes (paper Sec. 3.1, 3.2 and App. A).

Fluid: D3Q27, velocities in the order listed in App. A, weights by speed class from the
list in Sec. 3.1 (centre 8/27, face 2/27, edge 1/54, corner 1/216); App. A repeats the
list with the edge weight misprinted as 8/27, which would make the weights sum to 4.33.
Lattice sound speed c_s^2 = 1/3 (dx/dt = sqrt(3) c_s with dx = dt = 1).

Magnetic: D3Q7 with W = 1/4 (rest) and 1/8 (faces). Node coincidence 2C = sqrt(3) c_s
(Sec. 3.2) gives C = 1/2, C^2 = 1/4. The paper gives no order for the seven directions;
this oracle uses rest, -x, -y, -z, +x, +y, +z.
"""

import torch

DT = torch.float64

CX = [0, -1, 0, 0, -1, -1, -1, -1, 0, 0, -1, -1, -1, -1, 1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1]
CY = [0, 0, -1, 0, -1, 1, 0, 0, -1, -1, -1, -1, 1, 1, 0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1]
CZ = [0, 0, 0, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1]

C = torch.tensor([CX, CY, CZ], dtype=DT).T.contiguous()          # (27, 3)
Q = 27
CS2 = 1.0 / 3.0

_W_BY_SPEED2 = {0: 8.0 / 27.0, 1: 2.0 / 27.0, 2: 1.0 / 54.0, 3: 1.0 / 216.0}
W = torch.tensor([_W_BY_SPEED2[int(s)] for s in (C * C).sum(1)], dtype=DT)   # (27,)

XI = torch.tensor([[0, 0, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1],
                   [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=DT)  # (7, 3)
M7 = 7
C2 = 0.25
WM = torch.tensor([0.25] + [0.125] * 6, dtype=DT)


def opposite(i: int) -> int:
    """Index of -c_i in the App. A listing."""
    ci = C[i]
    for j in range(Q):
        if torch.equal(C[j], -ci):
            return j
    raise AssertionError


def omega_fluid(nu: float) -> float:
    """1/omega = nu / c_s^2 + 1/2 (Sec. 3.1, trapezoidal variable change)."""
    return 1.0 / (nu / CS2 + 0.5)


def omega_magnetic(eta: float) -> float:
    """1/omega_B = eta / C^2 + 1/2 (Sec. 3.2)."""
    return 1.0 / (eta / C2 + 0.5)


# ------------------------------------------------------------------ lattice variants
# The paper runs D3Q27 (fluid) with D3Q7 (magnetic). Sec. 4.3 reports runs with D3Q15 and D3Q27
# magnetic lattices (no significant gain), and the D3Q19 fluid set is the usual lower-connectivity
# alternative of the lattice figure of Sec. 3.1. The paper fixes neither the order of these sets
# nor the magnetic weights; the readings used here:
# * D3Q19 (fluid): the App. A listing without its eight corners (directions 0..9 and 14..22), so
#   the opposite of direction i <= 9 is i + 9; weights 1/3, 1/18, 1/36 by speed class, the D3Q19
#   set with the same c_s^2 = 1/3.
# * D3Q15 and D3Q27 (magnetic): node coincidence (Sec. 3.2) fixes C^2 = 1/4 for any magnetic
#   set, so its weights need sum W = 1 and sum W xi xi = C^2 I. The moving weights of the fluid
#   set with the same velocities scaled by C^2 / c_s^2 = 3/4, the rest weight taking the
#   remainder, meet both and keep that set's fourth-order isotropy
#   sum W xi_x^4 = 3 sum W xi_x^2 xi_y^2 (for D3Q15 they are the only isotropic choice):
#   D3Q15 rest 5/12, faces 1/12, corners 1/96; D3Q27 rest 17/36, faces 1/18, edges 1/72,
#   corners 1/288. Order of D3Q15: rest, -x, -y, -z, the four corners with xi_x = -1
#   ((-1,-1,-1), (-1,-1,1), (-1,1,-1), (-1,1,1)), then the opposites of those seven in the same
#   order (the opposite of i <= 7 is i + 7), which extends the D3Q7 order (rest, -x, -y, -z,
#   +x, +y, +z). Magnetic D3Q27 takes the App. A order.

class Lattice:
    """A velocity set: vectors c (q, 3), weights w (q,), the index of each opposite."""

    def __init__(self, name, c, w):
        self.name = name
        self.c = c
        self.w = w
        self.q = c.shape[0]
        self.opp = [next(j for j in range(self.q) if torch.equal(c[j], -c[i])) for i in range(self.q)]


def _by_speed(c, table):
    return torch.tensor([table[int(s)] for s in (c * c).sum(1)], dtype=DT)


_Q19 = list(range(10)) + list(range(14, 23))
C19 = C[_Q19].contiguous()
W19 = _by_speed(C19, {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0})

_XI15_HALF = [[-1, 0, 0], [0, -1, 0], [0, 0, -1], [-1, -1, -1], [-1, -1, 1], [-1, 1, -1], [-1, 1, 1]]
XI15 = torch.tensor([[0, 0, 0]] + _XI15_HALF + [[-a for a in v] for v in _XI15_HALF], dtype=DT)
WM15 = _by_speed(XI15, {0: 5.0 / 12.0, 1: 1.0 / 12.0, 3: 1.0 / 96.0})
XI27 = C.clone()
WM27 = _by_speed(XI27, {0: 17.0 / 36.0, 1: 1.0 / 18.0, 2: 1.0 / 72.0, 3: 1.0 / 288.0})

FLUID_LATTICES = {"d3q27": Lattice("d3q27", C, W), "d3q19": Lattice("d3q19", C19, W19)}
MAGNETIC_LATTICES = {"d3q7": Lattice("d3q7", XI, WM), "d3q15": Lattice("d3q15", XI15, WM15),
                     "d3q27": Lattice("d3q27", XI27, WM27)}
