"""The step of oracle.scheme evaluated in x87 extended precision (numpy longdouble, 64-bit
significand, unit roundoff 5.4e-20) -- TEST INFRASTRUCTURE ONLY.

The FP64 oracle carries full population values f ~ w_i; the physics lives in departures from
the rest state that can be 1e-3..1e-4 of that size, so its own rounding is amplified relative to
the quantities being compared, and the flow amplifies it further over many steps. This module
runs the same definition with ~2000x smaller rounding, which (a) measures the FP64 oracle's
floor and (b) serves as the reference for FP64 parity. It follows the paper passages named in
oracle.scheme; the fluid collision uses the exact closed form of the central-moment collision or
of its BGK limit (pinned equal to the T-matrix definition in tests/test_oracle_collision_current.py), the
equilibrium the D1Q3 product form (pinned equal to App. A's Hermite expansion), and J the
3x3 system of Sec. 3.2 solved by Cramer's rule (numpy's solver has no extended precision).
"""

from __future__ import annotations

import numpy as np

from . import lattice as _lat

LD = np.longdouble
C = _lat.C.numpy().astype(LD)                  # (27, 3), exact integers
XI = _lat.XI.numpy().astype(LD)                # (7, 3)
_W_BY_SPEED2 = {0: LD(8) / LD(27), 1: LD(2) / LD(27), 2: LD(1) / LD(54), 3: LD(1) / LD(216)}
W = np.array([_W_BY_SPEED2[int(s)] for s in (C * C).sum(1)], dtype=LD)
WM = np.array([LD(1) / LD(4)] + [LD(1) / LD(8)] * 6, dtype=LD)
CS2 = LD(1) / LD(3)
C2 = LD(1) / LD(4)


def _ld(t):
    if t is None:
        return None
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    return a.astype(LD)


class Params:
    def __init__(self, p):
        """From an oracle.scheme.Params."""
        self.nu, self.eta, self.d_i = LD(p.nu), LD(p.eta), LD(p.d_i)
        self.b0 = np.array(p.b0, dtype=LD)
        self.jmode = p.jmode
        self.omega = LD(1) / (self.nu / CS2 + LD(0.5))
        self.omega_b = LD(1) / (self.eta / C2 + LD(0.5))
        self.F = _ld(p.force_u)
        self.S = _ld(p.force_b)
        self.collision = p.collision
        self.magnetic = p.magnetic
        if self.collision not in ("central", "bgk") or self.magnetic not in ("hall", "emhd"):
            raise ValueError((self.collision, self.magnetic))


def _phi(c, u):
    """D1Q3 equilibrium factor for velocity component c in {-1, 0, 1}."""
    return np.where(c == 0, LD(2) / LD(3) - u * u, LD(0.5) * (CS2 + u * u + c * u))


def f_mhd_eq(rho, U, B):
    out = np.empty((27,) + rho.shape, dtype=LD)
    for i in range(27):
        out[i] = rho * _phi(C[i, 0], U[0]) * _phi(C[i, 1], U[1]) * _phi(C[i, 2], U[2])
    b2 = (B * B).sum(0)
    for i in range(27):
        cb = C[i, 0] * B[0] + C[i, 1] * B[1] + C[i, 2] * B[2]
        c2 = (C[i] * C[i]).sum()
        # (w/2c_s^4) M:(cc - c_s^2 I), M = |B|^2/2 I - BB:  M:cc = |B|^2/2 |c|^2 - (c.B)^2,
        # tr M = |B|^2/2
        out[i] += W[i] / (2 * CS2 * CS2) * (LD(0.5) * b2 * c2 - cb * cb - CS2 * LD(0.5) * b2)
    return out


def _h(p, c, u):
    if p == 0:
        return np.where(c == 0, LD(1) - u * u, LD(0.5) * (u * u + c * u))
    if p == 1:
        return np.where(c == 0, LD(-2) * u, u + LD(0.5) * c)
    return np.where(c == 0, LD(-1) + 0 * u, LD(0.5) + 0 * u)


def _unit(U, p):
    out = np.empty((27,) + U[0].shape, dtype=LD)
    for i in range(27):
        out[i] = _h(p[0], C[i, 0], U[0]) * _h(p[1], C[i, 1], U[1]) * _h(p[2], C[i, 2], U[2])
    return out


_PAIRS = {(0, 0): (2, 0, 0), (1, 1): (0, 2, 0), (2, 2): (0, 0, 2),
          (0, 1): (1, 1, 0), (0, 2): (1, 0, 1), (1, 2): (0, 1, 1)}
_FIRST = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def _cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _solve3(A, r):
    """Cramer's rule for A (3, 3, ...) x = r (3, ...)."""
    def det(m):
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    d = det(A)
    out = []
    for col in range(3):
        m = [[(r[row] if k == col else A[row][k]) for k in range(3)] for row in range(3)]
        out.append(det(m) / d)
    return np.stack(out)


def _current(p: Params, U, B, Lam):
    if p.jmode == "moment":
        z = np.zeros_like(B[0])
        one = np.ones_like(B[0])
        k = 2 * p.d_i * p.omega_b / C2
        A = [[one, k * B[2], -k * B[1]], [-k * B[2], one, k * B[0]], [k * B[1], -k * B[0], one]]
        del z
        A0 = np.stack([Lam[1, 2] - Lam[2, 1], Lam[2, 0] - Lam[0, 2], Lam[0, 1] - Lam[1, 0]])
        rhs = -(p.omega_b / C2) * (A0 - 2 * _cross(U, B))
        return _solve3(A, rhs)
    d = lambda f, axis: LD(0.5) * (np.roll(f, -1, axis=2 - axis) - np.roll(f, 1, axis=2 - axis))  # noqa: E731
    return np.stack([d(B[2], 1) - d(B[1], 2), d(B[0], 2) - d(B[2], 0), d(B[1], 0) - d(B[0], 1)])


def step(f, g, p: Params, nsteps=1):
    """f (27, nz, ny, nx), g (7, 3, nz, ny, nx) longdouble; returns the state after nsteps."""
    for _ in range(nsteps):
        rho = f.sum(0)
        mom = np.einsum("i...,ia->a...", f, C)
        if p.F is not None:
            mom = mom + LD(0.5) * p.F
        U = mom / rho
        B = g.sum(0)
        if p.S is not None:
            B = B + LD(0.5) * p.S
        Lam = np.einsum("ia,ib...->ab...", XI, g)
        Um = np.zeros_like(U) if p.magnetic == "emhd" else U
        J = _current(p, Um, B, Lam)
        f0 = f_mhd_eq(rho, U, B)
        if p.collision == "bgk":
            fs = f0 + (1 - p.omega) * (f - f0)
            if p.F is not None:
                for a, pp in enumerate(_FIRST):
                    fs += (1 - p.omega / 2) * p.F[a] * _unit(U, pp)
        else:
            d = f - f0
            cb = C.T.reshape(3, 27, *([1] * U[0].ndim)) - U[:, None]
            K = np.einsum("ai...,bi...,i...->ab...", cb, cb, d)
            tr = (K[0, 0] + K[1, 1] + K[2, 2]) / 3
            fs = f0.copy()
            for (a, b), pp in _PAIRS.items():
                Pab = K[a, b] - (tr if a == b else 0)
                fs += (1 - p.omega) * Pab * _unit(U, pp)
            if p.F is not None:
                for a, pp in enumerate(_FIRST):
                    fs += LD(0.5) * p.F[a] * _unit(U, pp)
        V = Um - p.d_i * J
        xv = np.einsum("ib,b...->i...", XI, V)
        xb = np.einsum("ib,b...->i...", XI, B)
        geq = WM.reshape(7, 1, *([1] * U[0].ndim)) * (B[None] + (xv[:, None] * B[None] - xb[:, None] * V[None]) / C2)
        gs = g - p.omega_b * (g - geq)
        if p.S is not None:
            gs = gs + (1 - p.omega_b / 2) * WM.reshape(7, 1, *([1] * U[0].ndim)) * p.S[None]
        f = np.stack([np.roll(fs[i], (int(C[i, 2]), int(C[i, 1]), int(C[i, 0])), axis=(0, 1, 2))
                      for i in range(27)])
        g = np.stack([np.roll(gs[i], (int(XI[i, 2]), int(XI[i, 1]), int(XI[i, 0])), axis=(1, 2, 3))
                      for i in range(7)])
    return f, g


def init_state(p: Params, u, b, grad_u=None, grad_b=None, noneq=True):
    """The initial state of oracle.scheme.init_state, in extended precision; the first-order
    non-equilibrium fluid part is assembled from the unit central-moment distributions."""
    u, b = _ld(u), _ld(b)
    gu, gb = _ld(grad_u), _ld(grad_b)
    B = b + p.b0.reshape(3, 1, 1, 1)
    rho = np.ones_like(u[0])
    f = f_mhd_eq(rho, u, B)
    if noneq and gu is not None:
        s = gu + np.swapaxes(gu, 0, 1)
        div = gu[0, 0] + gu[1, 1] + gu[2, 2]
        for (a, bb), pp in _PAIRS.items():
            Pab = -(CS2 / p.omega) * (s[a, bb] - (LD(2) / 3 * div if a == bb else 0))
            f = f + Pab * _unit(u, pp)
    if p.F is not None:
        for a, pp in enumerate(_FIRST):
            f = f - LD(0.5) * p.F[a] * _unit(u, pp)
    J = np.zeros_like(u) if gb is None else np.stack(
        [gb[1, 2] - gb[2, 1], gb[2, 0] - gb[0, 2], gb[0, 1] - gb[1, 0]])
    V = (np.zeros_like(u) if p.magnetic == "emhd" else u) - p.d_i * J
    xv = np.einsum("ib,b...->i...", XI, V)
    xb = np.einsum("ib,b...->i...", XI, B)
    wm = WM.reshape(7, 1, 1, 1, 1)
    g = wm * (B[None] + (xv[:, None] * B[None] - xb[:, None] * V[None]) / C2)
    if noneq and gb is not None:
        xg = np.einsum("ia,ab...->ib...", XI, gb)
        g = g - wm * xg / p.omega_b
    if p.S is not None:
        g = g - LD(0.5) * wm * p.S[None]
    return f, g


def rest_state(p: Params, shape):
    z = np.zeros((3,) + tuple(shape), dtype=LD)
    B = z + p.b0.reshape(3, 1, 1, 1)
    f = f_mhd_eq(np.ones(shape, dtype=LD), z, B)
    g = WM.reshape(7, 1, 1, 1, 1) * B[None]
    return f, g
