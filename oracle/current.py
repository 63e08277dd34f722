"""Electric current density J (paper Sec. 3.2, eqs. LB_density_current, soe_current_density,
App. B) and the divergence diagnostic (eq. LB_B_div).

Moment route (the paper's): the non-equilibrium part of the magnetic first moment gives
J_g = -eps_{abg} (w_B / C^2) (Lambda_ab - Lambda0_ab). Because Lambda0 itself contains J
through the Hall velocity U - alpha_H J, this is the linear 3x3 system
    (I + (2 alpha_H w_B / C^2) M(B)) J = -(w_B / C^2) J0,
with M(B) and J0 as printed in Sec. 3.2. The printed system omits the factor -w_B / C^2 on
the right-hand side; it is restored here so that the system is the same as the defining
relation above (App. B carries the equivalent factor -1/(2 alpha_H) after dividing through
by 2 alpha_H w_B / C^2). The oracle solves the 3x3 system directly.

Stencil route (an alternative the method admits): J = curl B by second-order central
differences of B on the six face neighbours, periodic grid.
"""

import torch

from .lattice import C2


def levi_civita_contract(Lam):
    """A_g = eps_{g a b} Lambda_ab: (Lyz - Lzy, Lzx - Lxz, Lxy - Lyx)."""
    return torch.stack([Lam[1, 2] - Lam[2, 1], Lam[2, 0] - Lam[0, 2], Lam[0, 1] - Lam[1, 0]])


def cross(a, b):
    return torch.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def m_matrix(B):
    """M(B) of eq. soe_objects, shape (3, 3, n)."""
    z = torch.zeros_like(B[0])
    return torch.stack([torch.stack([z, B[2], -B[1]]),
                        torch.stack([-B[2], z, B[0]]),
                        torch.stack([B[1], -B[0], z])])


def j0_vector(Lam, U, B):
    """J0 of eq. soe_objects."""
    return levi_civita_contract(Lam) - 2.0 * cross(U, B)


def current_moment(Lam, U, B, alpha_h, omega_b):
    """Solve (I + 2 alpha_H w_B / C^2 M) J = -(w_B / C^2) J0 node by node. Shapes (3,3,n),(3,n)."""
    n = B.shape[1]
    A = torch.eye(3, dtype=B.dtype).unsqueeze(-1).expand(3, 3, n) \
        + (2.0 * alpha_h * omega_b / C2) * m_matrix(B)
    rhs = -(omega_b / C2) * j0_vector(Lam, U, B)
    return torch.linalg.solve(A.permute(2, 0, 1), rhs.T.unsqueeze(-1)).squeeze(-1).T


def current_stencil(B):
    """Central-difference curl of B (3, nz, ny, nx), periodic. Axis order z, y, x."""
    def d(f, axis):  # derivative along lattice axis 0=x, 1=y, 2=z
        dim = 3 - axis
        return 0.5 * (torch.roll(f, -1, dims=dim) - torch.roll(f, 1, dims=dim))
    Bx, By, Bz = B[0:1], B[1:2], B[2:3]
    jx = d(Bz, 1) - d(By, 2)
    jy = d(Bx, 2) - d(Bz, 0)
    jz = d(By, 0) - d(Bx, 1)
    return torch.cat([jx, jy, jz], dim=0)


def divergence_moment(Lam, omega_b):
    """div B ~ -(w_B / C^2) Tr Lambda (eq. LB_B_div)."""
    return -(omega_b / C2) * (Lam[0, 0] + Lam[1, 1] + Lam[2, 2])
