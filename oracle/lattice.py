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
