"""Global diagnostics: energies, cross-helicity, current, divergence, invariants (paper Sec.
4.4: mean energies, <|J|^2>, dissipation; eq. LB_B_div) and shell energy spectra (Sec. 4.4).

Reduction slots, in order:
  0 E_kin = 1/2 <|u|^2>            1 E_mag = 1/2 <|B - b0|^2>      2 H_c = <u . (B - b0)>
  3 <|J|^2>                        4 max |div B|                   5 rms div B
  6 max |u|                        7 rms (rho - 1)                 8 nodes with a non-finite value
  9 sum rho                        10..12 sum rho u                13..15 sum B
div B is the moment estimate -(w_B / C^2) Tr Lambda.

Spectrum of a vector field v on an n^3 grid: E(s) = 1/2 sum_{round(|k|) = s} |v_hat(k)|^2 with
v_hat = DFT(v) / n^3 and k the signed integer wavevector; by Parseval sum_s E(s) = 1/2 <|v|^2>.

Dissipation spectrum (the summand of D(k) in Sec. 4.4, eq. mhd_en_trans, without the factor nu
or eta): D(s) = sum_{round(|k|) = s} |q(k)|^2 |v_hat(k)|^2, with q_a = 2 pi k_a / n_a the
wavevector in inverse cells; sum_s D(s) = <|grad v|^2> of the grid's trigonometric interpolant,
which is <|curl v|^2> when v is solenoidal. The dissipation rate of the energy 1/2 <|u|^2 + |B|^2>
is then nu sum_s D_u(s) + eta sum_s D_B(s).

Energy transfer (the summands of the flux S_MHD(k) in Sec. 4.4, per shell s):
  T_adv(s) = sum Re[u_hat* . F(U . grad U)],  T_lor(s) = -sum Re[u_hat* . F(J x B)],
  T_ind(s) = -sum Re[B_hat* . F(curl(U x B))],
so that S_MHD(k) = sum_{s < k} (T_adv + T_lor + T_ind) and, for incompressible MHD without the
Hall and pressure terms, d/dt sum_{s < k} E(s) = -S_MHD(k) - D(k). The Hall term of the induction
equation, -alpha_H curl(J x B), which the paper's flux leaves out, transfers
T_hall(s) = +alpha_H sum Re[B_hat* . F(curl(J x B))]; it conserves the energy (its sum over all
shells is alpha_H <J . (J x B)> = 0 for J = curl B). Derivatives are spectral with
q_a = 2 pi k_a / n_a, except that q_a = 0 on the Nyquist index of an even axis (that mode's
derivative is not a real field). Products are formed node by node on the grid.
"""

import math

import numpy as np
import torch

from . import scheme

NRED = 16


def reductions(st, p):
    rho, U, B, J, divb = scheme.fields(st, p)
    b0 = torch.tensor(p.b0, dtype=torch.float64).view(3, 1, 1, 1)
    bb = B - b0
    bad = ~(torch.isfinite(st.f).all(0) & torch.isfinite(st.g).all(0).all(0))
    out = torch.zeros(NRED, dtype=torch.float64)
    out[0] = 0.5 * (U * U).sum(0).mean()
    out[1] = 0.5 * (bb * bb).sum(0).mean()
    out[2] = (U * bb).sum(0).mean()
    out[3] = (J * J).sum(0).mean()
    out[4] = divb.abs().max()
    out[5] = (divb * divb).mean().sqrt()
    out[6] = (U * U).sum(0).sqrt().max()
    out[7] = ((rho - 1.0) ** 2).mean().sqrt()
    out[8] = bad.sum()
    out[9] = rho.sum()
    out[10:13] = (rho.unsqueeze(0) * U).sum((1, 2, 3))
    out[13:16] = B.sum((1, 2, 3))
    return out


def shell_index(shape):
    """round(|k|) for every DFT index of a (nz, ny, nx) grid (signed integer k per axis)."""
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    kk = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    return np.floor(kk + 0.5).astype(np.int64)


def spectrum(v, nshells):
    """Shell energy spectrum of a (3, nz, ny, nx) real field; shells 0..nshells-1."""
    arr = v.detach().cpu().numpy() if torch.is_tensor(v) else np.asarray(v)
    n = arr[0].size
    e = np.zeros(nshells)
    s = shell_index(arr.shape[1:])
    for b in range(3):
        vh = np.fft.fftn(arr[b]) / n
        e += np.bincount(s.ravel(), weights=0.5 * np.abs(vh.ravel()) ** 2, minlength=nshells)[:nshells]
    return e


def dissipation_spectrum(v, nshells):
    """Shell dissipation spectrum of a (3, nz, ny, nx) real field; shells 0..nshells-1."""
    arr = v.detach().cpu().numpy() if torch.is_tensor(v) else np.asarray(v)
    nz, ny, nx = arr.shape[1:]
    n = arr[0].size
    qz = 2 * np.pi * np.fft.fftfreq(nz, 1.0 / nz) / nz
    qy = 2 * np.pi * np.fft.fftfreq(ny, 1.0 / ny) / ny
    qx = 2 * np.pi * np.fft.fftfreq(nx, 1.0 / nx) / nx
    q2 = qz[:, None, None] ** 2 + qy[None, :, None] ** 2 + qx[None, None, :] ** 2
    d = np.zeros(nshells)
    s = shell_index(arr.shape[1:])
    for b in range(3):
        vh = np.fft.fftn(arr[b]) / n
        d += np.bincount(s.ravel(), weights=(q2 * np.abs(vh) ** 2).ravel(), minlength=nshells)[:nshells]
    return d


def derivative_wavenumbers(n):
    """2 pi k / n for the signed DFT index k of an axis of n nodes; 0 at the Nyquist index."""
    q = 2.0 * np.pi * np.fft.fftfreq(n, 1.0 / n) / n
    if n % 2 == 0:
        q[n // 2] = 0.0
    return q


def energy_transfer(U, B, J, nshells, d_i=None):
    """(T_adv, T_lor, T_ind), each (nshells,), of (3, nz, ny, nx) real fields U, B and J; with
    d_i (alpha_H) given, T_hall is appended."""
    U, B, J = [x.detach().cpu().numpy() if torch.is_tensor(x) else np.asarray(x) for x in (U, B, J)]
    nz, ny, nx = U.shape[1:]
    ncell = U[0].size
    Q = (derivative_wavenumbers(nx)[None, None, :], derivative_wavenumbers(ny)[None, :, None],
         derivative_wavenumbers(nz)[:, None, None])
    shell = shell_index(U.shape[1:]).ravel()
    hat = lambda v: np.fft.fftn(v) / ncell  # noqa: E731

    def binned(values):
        return np.bincount(shell, weights=values.ravel(), minlength=nshells)[:nshells]

    Uh = [hat(U[b]) for b in range(3)]
    Bh = [hat(B[b]) for b in range(3)]
    # (U . grad) U with grad U_b = inverse DFT of i q_a u_hat_b
    adv = [sum(U[a] * np.real(np.fft.ifftn(1j * Q[a] * np.fft.fftn(U[b]))) for a in range(3)) for b in range(3)]
    lor = np.cross(J, B, axis=0)
    W = np.cross(U, B, axis=0)
    Wh = [hat(W[b]) for b in range(3)]
    t_adv = sum(binned(np.real(np.conj(Uh[b]) * hat(adv[b]))) for b in range(3))
    t_lor = -sum(binned(np.real(np.conj(Uh[b]) * hat(lor[b]))) for b in range(3))
    def curl_hat(Vh, b):
        c, d = (b + 1) % 3, (b + 2) % 3
        return 1j * (Q[c] * Vh[d] - Q[d] * Vh[c])

    t_ind = -sum(binned(np.real(np.conj(Bh[b]) * curl_hat(Wh, b))) for b in range(3))
    if d_i is None:
        return t_adv, t_lor, t_ind
    Lh = [hat(lor[b]) for b in range(3)]
    t_hall = d_i * sum(binned(np.real(np.conj(Bh[b]) * curl_hat(Lh, b))) for b in range(3))
    return t_adv, t_lor, t_ind, t_hall


def max_shell(shape):
    nz, ny, nx = shape
    return int(math.floor(math.sqrt((nz // 2) ** 2 + (ny // 2) ** 2 + (nx // 2) ** 2) + 0.5)) + 1


def turbulence_summary(U, B, nu, eta, b0=(0.0, 0.0, 0.0), nshells=None):
    """Mean-flow quantities of the paper's turbulence runs (Sec. 4.4) from node fields U, B
    (3, nz, ny, nx): E_kin = 1/2 <|u|^2>, E_mag = 1/2 <|B - b0|^2>, the dissipation rate
    eps = nu <|grad u|^2> + eta <|grad B|^2> (sums of the dissipation spectra), U = the r.m.s.
    velocity <|u|^2>^(1/2), the integral length L = 2 pi int E_u(k)/k dk / int E_u(k) dk over
    shells k = 1..nshells-1 with the box of n cells taken as 2 pi (so L in cells is
    n sum_k E_u(k)/k / sum_k E_u(k), n the largest axis), and Re = U L / nu."""
    arr = U.detach().cpu().numpy() if torch.is_tensor(U) else np.asarray(U)
    barr = B.detach().cpu().numpy() if torch.is_tensor(B) else np.asarray(B)
    n = max(arr.shape[1:])
    nshells = nshells or n // 2 + 1
    e_kin = 0.5 * float((arr ** 2).sum(0).mean())
    bf = barr - np.asarray(b0, dtype=np.float64).reshape(3, 1, 1, 1)
    e_mag = 0.5 * float((bf ** 2).sum(0).mean())
    eps = nu * float(dissipation_spectrum(arr, nshells).sum()) + eta * float(dissipation_spectrum(barr, nshells).sum())
    eu = spectrum(arr, nshells)[1:]
    k = np.arange(1, nshells, dtype=np.float64)
    scale = n * float((eu / k).sum() / eu.sum()) if eu.sum() > 0 else 0.0
    u_rms = math.sqrt(2.0 * e_kin)
    return {"E_kin": e_kin, "E_mag": e_mag, "eps": eps, "u_rms": u_rms, "integral_scale": scale,
            "Re": u_rms * scale / nu}
