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


def emhd_frequency(alpha_h: float, k: float, b0: float) -> float:
    """Whistler frequency of the electron-MHD induction equation (Sec. 6: the magnetic
    equilibrium without the bulk velocity), w = alpha_H b0 k^2.

    With V = -alpha_H J the magnetic scheme solves dB/dt = -alpha_H curl(J x B) + eta lap B. For
    B = b0 z_hat + b(z, t), b perpendicular to z: J = curl b lies in the plane, J x b is along z
    and depends on z only (its curl vanishes), and J x (b0 z_hat) = b0 d_z b, so
    d_t b_x = alpha_H b0 d_z^2 b_y + eta d_z^2 b_x, d_t b_y = -alpha_H b0 d_z^2 b_x + eta d_z^2 b_y.
    b = a exp(-eta k^2 t) (sin(k z - w t), cos(k z - w t), 0) solves this exactly for
    w = alpha_H b0 k^2, whatever the fluid does."""
    return alpha_h * b0 * k * k


def emhd_wave(nz: int, t: float, amp: float, b0: float, eta: float, alpha_h: float, mode: int = 1):
    """Exact electron-MHD field B(z, t) (includes b0 along z) on z = 0..nz-1: (3, nz)."""
    k = 2.0 * math.pi * mode / nz
    w = emhd_frequency(alpha_h, k, b0)
    z = torch.arange(nz, dtype=torch.float64)
    ph = k * z - w * t
    damp = amp * math.exp(-eta * k * k * t)
    b = torch.stack([damp * torch.sin(ph), damp * torch.cos(ph), torch.zeros_like(ph)])
    b[2] += b0
    return b

