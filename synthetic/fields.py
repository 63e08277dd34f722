"""Fourier-mode vector fields: the seeded initial conditions and forcing fields.

A field is  f(x) = sum_k 2 Re[ v_k exp(2 pi i k . x / n) ]  over a list of half-space
wavevectors k (integer, one representative of each +-k pair), with complex 3-vectors v_k.
Its mean square is  <|f|^2> = sum_k 2 |v_k|^2  whenever no two listed modes alias on the
grid (n > 2 max|k_a| on every axis), so the rms target is met exactly and independently of
the grid size.

Recipes (see the design notes for the workloads they stand in for):
  * shell_field: random-phase field, solenoidal on cubic grids (k . v_k = 0), with equal energy in each shell
    round(|k|) in [kmin, kmax] (or |k| <= kmax with ``select="radius"``), drawn with
    numpy's PCG64 generator from a seed, rescaled to a given rms of |f|.
  * wave_field: the circularly polarised plane wave a (sin kz, cos kz, 0).
  * xia_field: the three-mode Beltrami field of the paper's validation runs (Sec. 4.1).
  * orszag_tang: the Orszag-Tang vortex velocity and magnetic field of the paper's comparison
    with a pseudo-spectral code and of its Hall-MHD runs (Sec. 4.4, Sec. 5).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class ModeField:
    """k: (M, 3) int64 wavevector indices (kx, ky, kz); v: (M, 3) complex128 amplitudes."""

    k: np.ndarray
    v: np.ndarray

    def __post_init__(self):
        assert self.k.ndim == 2 and self.k.shape[1] == 3
        assert self.v.shape == self.k.shape

    @property
    def mean_square(self) -> float:
        return float(2.0 * np.sum(np.abs(self.v) ** 2))

    @property
    def rms(self) -> float:
        return math.sqrt(self.mean_square)


def _is_half_space(k) -> bool:
    kx, ky, kz = k
    return kz > 0 or (kz == 0 and ky > 0) or (kz == 0 and ky == 0 and kx > 0)


def half_space_wavevectors(kmin: float, kmax: float, select: str = "shell") -> np.ndarray:
    """Half-space integer wavevectors in lexicographic (kz, ky, kx) order.

    select="shell": kmin <= round(|k|) <= kmax (round half up: n - 1/2 <= |k| < n + 1/2).
    select="radius": 0 < |k| <= kmax (kmin ignored beyond excluding k = 0).
    """
    r = int(math.ceil(kmax + 1))
    out = []
    for kz in range(-r, r + 1):
        for ky in range(-r, r + 1):
            for kx in range(-r, r + 1):
                if not _is_half_space((kx, ky, kz)):
                    continue
                kk = math.sqrt(kx * kx + ky * ky + kz * kz)
                if select == "shell":
                    n = int(math.floor(kk + 0.5))
                    ok = kmin <= n <= kmax
                elif select == "radius":
                    ok = 0 < kk <= kmax + 1e-12
                else:
                    raise ValueError(select)
                if ok:
                    out.append((kx, ky, kz))
    return np.asarray(out, dtype=np.int64).reshape(-1, 3)


def shell_field(seed: int, kmin: int, kmax: int, rms: float, select: str = "shell") -> ModeField:
    """Random-phase solenoidal field, flat shell spectrum, rms of |f| equal to ``rms``."""
    k = half_space_wavevectors(kmin, kmax, select)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((k.shape[0], 3, 2))
    v = (g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0)
    kf = k.astype(np.float64)
    k2 = np.sum(kf * kf, axis=1)
    v = v - kf * (np.sum(kf * v, axis=1) / k2)[:, None]          # solenoidal: k . v = 0
    shell = np.floor(np.sqrt(k2) + 0.5).astype(np.int64)
    for n in np.unique(shell):                                    # equal energy per shell
        m = shell == n
        v[m] /= math.sqrt(np.sum(np.abs(v[m]) ** 2))
    f = ModeField(k, v)
    return scaled(f, rms / f.rms)


def wave_field(amp: float, kz: int = 1) -> ModeField:
    """u = amp (sin(2 pi kz z / n), cos(2 pi kz z / n), 0)."""
    k = np.array([[0, 0, kz]], dtype=np.int64)
    v = np.array([[-0.5j * amp, 0.5 * amp, 0.0]], dtype=np.complex128)
    return ModeField(k, v)


def xia_field(u0: float, a: float = 0.3, b: float = 0.2, c: float = 0.1, kidx: int = 2) -> ModeField:
    """Three-mode Beltrami velocity of the paper's validation initial condition (Sec. 4.1).

    ux = u0 (b sin(q z) + a cos(q y)), uy = u0 (b cos(q z) + c sin(q x)),
    uz = u0 (c cos(q x) + a sin(q y)), with q = 2 pi kidx / n.
    """
    k = np.array([[0, 0, kidx], [0, kidx, 0], [kidx, 0, 0]], dtype=np.int64)
    v = 0.5 * u0 * np.array([[-1j * b, b, 0.0],
                             [a, 0.0, -1j * a],
                             [0.0, -1j * c, c]], dtype=np.complex128)
    return ModeField(k, v)


def orszag_tang(u_amp: float, b_amp: float) -> tuple[ModeField, ModeField]:
    """Orszag-Tang vortex on a box of 2 pi per axis (Sec. 4.4), with X = 2 pi x / n per axis:

    u = u_amp (-2 sin Y, 2 sin X, 0),
    B = b_amp (-2 sin 2Y + sin Z, 2 sin X + sin Z, sin X + sin Y).

    Both are solenoidal; <|u|^2> = 4 u_amp^2, <|B|^2> = 6 b_amp^2, <u . B> = 2 u_amp b_amp.
    Uses sin t = 2 Re[(-i/2) e^{i t}] on the modes (1,0,0), (0,1,0), (0,2,0), (0,0,1).
    """
    h = -0.5j
    ku = np.array([[1, 0, 0], [0, 1, 0]], dtype=np.int64)
    vu = u_amp * np.array([[0.0, 2 * h, 0.0],
                           [-2 * h, 0.0, 0.0]], dtype=np.complex128)
    kb = np.array([[1, 0, 0], [0, 1, 0], [0, 2, 0], [0, 0, 1]], dtype=np.int64)
    vb = b_amp * np.array([[0.0, 2 * h, h],
                           [0.0, 0.0, h],
                           [-2 * h, 0.0, 0.0],
                           [h, h, 0.0]], dtype=np.complex128)
    return ModeField(ku, vu), ModeField(kb, vb)


def scaled(f: ModeField, s: float) -> ModeField:
    return ModeField(f.k.copy(), f.v * s)


def _spectrum_entries(f: ModeField, shape):
    """Full-DFT entries (index, value, signed k) for both members of every +-k pair."""
    nx, ny, nz = shape
    if f.k.size:
        kmax = np.max(np.abs(f.k), axis=0)
        if not (nx > 2 * kmax[0] and ny > 2 * kmax[1] and nz > 2 * kmax[2]):
            raise ValueError(f"grid {shape} aliases modes up to {kmax.tolist()}")
    ks = np.concatenate([f.k, -f.k], axis=0)
    vs = np.concatenate([f.v, np.conj(f.v)], axis=0)
    idx = np.stack([ks[:, 2] % nz, ks[:, 1] % ny, ks[:, 0] % nx], axis=1)
    return idx, vs, ks


def evaluate(f: ModeField, shape, device="cpu", gradient=True):
    """Sample the field on an (nx, ny, nz) grid with torch (CPU or GPU).

    Returns (val, grad): val[b, z, y, x] = f_b; grad[a, b, z, y, x] = d f_b / d x_a
    (derivative direction first), both float64 torch tensors on ``device``; grad is None
    when ``gradient`` is False.
    """
    import torch

    nx, ny, nz = shape
    idx, vs, ks = _spectrum_entries(f, shape)
    n = np.array([nx, ny, nz], dtype=np.float64)
    lin = torch.as_tensor((idx[:, 0] * ny + idx[:, 1]) * nx + idx[:, 2], device=device)
    vals = torch.as_tensor(vs, device=device)                       # (2M, 3) complex
    scale = float(nx * ny * nz)

    def synth(coef):  # coef: (2M,) complex -> real field (nz, ny, nx)
        c = torch.zeros(nz * ny * nx, dtype=torch.complex128, device=device)
        c.index_put_((lin,), coef, accumulate=True)
        r = torch.fft.ifftn(c.view(nz, ny, nx)).real * scale
        return r

    val = torch.empty((3, nz, ny, nx), dtype=torch.float64, device=device)
    for b in range(3):
        val[b] = synth(vals[:, b])
    if not gradient:
        return val, None
    grad = torch.empty((3, 3, nz, ny, nx), dtype=torch.float64, device=device)
    ik = torch.as_tensor(1j * 2.0 * np.pi * ks / n[None, :], device=device)  # (2M, 3)
    for a in range(3):
        for b in range(3):
            grad[a, b] = synth(ik[:, a] * vals[:, b])
    return val, grad


def evaluate_numpy(f: ModeField, points: np.ndarray, shape, gradient=False):
    """Direct mode sum at given integer points (P, 3) = (x, y, z): returns (P, 3) values.

    Independent of the FFT path above; used to cross-check it and to sample large grids
    at a few points.
    """
    nx, ny, nz = shape
    n = np.array([nx, ny, nz], dtype=np.float64)
    ph = 2.0 * np.pi * (points.astype(np.float64) / n[None, :]) @ f.k.T.astype(np.float64)
    e = np.exp(1j * ph)                                             # (P, M)
    val = 2.0 * np.real(e @ f.v)
    if not gradient:
        return val
    ik = 1j * 2.0 * np.pi * f.k / n[None, :]                        # (M, 3)
    grad = np.stack([2.0 * np.real(e @ (ik[:, a:a + 1] * f.v)) for a in range(3)], axis=1)
    return val, grad
