"""Exact damped circularly polarised Hall-MHD wave (paper Sec. 4.1, after Xia & Yang),
written in lattice units.

For rho = 1, nu = eta, uniform field b0 along z and wavenumber k along z:
    u(z, t) = a exp(-nu k^2 t) (sin(k z - w t), cos(k z - w t), 0),   b = b0 z_hat + beta u,
with beta^2 + alpha_H k beta - 1 = 0, i.e. beta = -alpha_H k / 2 +- sqrt(alpha_H^2 k^2 / 4 + 1),
and w = -k b0 beta. This is the paper's relation w = -alpha k with eps_H k -> alpha_H k and the
field measured in units of b0. The velocity is a curl eigenfunction (curl u = k u), so every
nonlinear term of the incompressible equations vanishes and the wave is exact.
"""

import math

import torch


def beta(alpha_h: float, k: float, branch: int = +1) -> float:
    """Roots of beta^2 + alpha_H k beta - 1 = 0; branch +1 is the paper's alpha_+."""
    return -0.5 * alpha_h * k + branch * math.sqrt(0.25 * (alpha_h * k) ** 2 + 1.0)


def frequency(alpha_h: float, k: float, b0: float, branch: int = +1) -> float:
    return -k * b0 * beta(alpha_h, k, branch)


def wave(nz: int, t: float, amp: float, b0: float, nu: float, alpha_h: float, branch: int = +1,
         mode: int = 1):
    """Exact u(z, t), b(z, t) (full field, includes b0 along z) on z = 0..nz-1: (3, nz) each."""
    k = 2.0 * math.pi * mode / nz
    be = beta(alpha_h, k, branch)
    w = -k * b0 * be
    z = torch.arange(nz, dtype=torch.float64)
    ph = k * z - w * t
    damp = amp * math.exp(-nu * k * k * t)
    u = torch.stack([damp * torch.sin(ph), damp * torch.cos(ph), torch.zeros_like(ph)])
    b = be * u
    b[2] += b0
    return u, b
