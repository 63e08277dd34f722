"""Central-moment collision of the fluid populations (paper Sec. 3.1.2 and App. A).

Moments k = T^T f with the 27 column vectors T_j of polynomials in cbar = c - U; collision
k* = k - S (k - k^(0)) with S = diag[1,1,1,1, w x5, 1 x18]; back-transform f* = T^{-T} k*.

Basis reading: as printed, T_11, T_12, T_14, T_15 never contain the monomial cbar_x^2 cbar_z,
so T has rank 26 and cannot be inverted although the text calls it invertible. They are
read as the symmetric / antisymmetric pairs of the three mixed third-order monomials that
match T_10 and T_13:
    T_11 = cx^2 cy + cy cz^2,   T_12 = cx^2 cz + cy^2 cz,
    T_14 = cx^2 cy - cy cz^2,   T_15 = cx^2 cz - cy^2 cz.
The collision result does not depend on this choice: every moment outside T_4..T_8 relaxes
with rate 1 (or is conserved), so any invertible basis whose T_0..T_9 are the printed ones
gives the same f*.

Two routes are provided:
  * collide_T: the definition above with an explicit 27x27 solve per node. It is evaluated
    as f* = f0 + T^{-T} (k* - k0), the same quantity written so that rounding scales with
    the non-equilibrium part rather than with f itself.
  * collide_closed: the exact closed form that follows because only the five deviatoric
    second-order moments keep a non-equilibrium part: f* = f0 + (1 - w) sum_ab P_ab D^ab,
    where P is the deviatoric second central moment of f - f0 and D^ab are products of the
    1-D functions h_p whose central moments about U are (delta_p0, delta_p1, delta_p2).

Forcing (an extension: the paper simulates unforced turbulence): with the velocity shifted
by F/(2 rho), the pre-collision first central moments equal -F/2 and are set to +F/2 by the
collision, so each collision adds F to the momentum.
"""

import torch

from .equilibrium import f_mhd_eq
from .lattice import C


def _t_columns(cb, printed=False):
    """The 27 basis polynomials evaluated at cbar (n, 27, 3) -> (n, 27, 27) [node, i, j]."""
    x, y, z = cb[..., 0], cb[..., 1], cb[..., 2]
    x2, y2, z2 = x * x, y * y, z * z
    cols = [torch.ones_like(x), x, y, z, x * y, x * z, y * z, x2 - y2, x2 - z2, x2 + y2 + z2,
            x * y2 + x * z2]
    if printed:
        cols += [x * y2 + y * z2, x2 * y + y2 * z, x * y2 - x * z2, x * y2 - y * z2, x2 * y - y2 * z]
    else:
        cols += [x2 * y + y * z2, x2 * z + y2 * z, x * y2 - x * z2, x2 * y - y * z2, x2 * z - y2 * z]
    cols += [x * y * z, x2 * y2 + x2 * z2 + y2 * z2, x2 * y2 + x2 * z2 - y2 * z2, x2 * y2 - x2 * z2,
             x2 * y * z, x * y2 * z, x * y * z2, x * y2 * z2, x2 * y * z2, x2 * y2 * z, x2 * y2 * z2]
    return torch.stack(cols, dim=-1)


def t_matrix(U, printed=False):
    """T[n, i, j] = T_j(c_i - U_n) for U of shape (3, n)."""
    cb = C.unsqueeze(0) - U.T.unsqueeze(1)          # (n, 27, 3)
    return _t_columns(cb, printed)


def relaxation_rates(omega):
    """S = diag[1, 1, 1, 1, w, w, w, w, w, 1, ..., 1] (eq. collision_matrix)."""
    s = torch.ones(27, dtype=torch.float64)
    s[4:9] = omega
    return s


def collide_T(f, rho, U, B, omega, F=None, rates=None, chunk=8192):
    """Central-moment collision by the explicit moment transform. f: (27, n); U, B, F: (3, n)."""
    s = relaxation_rates(omega) if rates is None else rates
    f0 = f_mhd_eq(rho, U, B)
    out = torch.empty_like(f)
    n = f.shape[1]
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        T = t_matrix(U[:, lo:hi])                                   # (m, 27, 27)
        dk = torch.einsum("mij,im->mj", T, f[:, lo:hi] - f0[:, lo:hi])   # k - k0
        dks = (1.0 - s)[None, :] * dk                               # k* - k0
        if F is not None:
            dks[:, 1:4] = 0.5 * F[:, lo:hi].T                       # k*_{1..3} = F/2, k0 = 0
        x = torch.linalg.solve(T.transpose(1, 2), dks.unsqueeze(-1)).squeeze(-1)
        out[:, lo:hi] = f0[:, lo:hi] + x.T
    return out


def moments_to_dist(U, k, chunk=8192):
    """Populations x with T^T x = k node by node (the back-transform T^{-T}). U (3,n), k (n,27)."""
    n = k.shape[0]
    out = torch.empty((27, n), dtype=k.dtype)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        T = t_matrix(U[:, lo:hi])
        out[:, lo:hi] = torch.linalg.solve(T.transpose(1, 2), k[lo:hi].unsqueeze(-1)).squeeze(-1).T
    return out


def _h(p, c, u):
    """1-D functions on {-1, 0, 1} with central moments about u equal to delta_{p,q}, q=0,1,2.

    c: (27, 1) lattice components, u: (n,) -> (27, n)."""
    one = torch.ones_like(c * u)
    if p == 0:
        return torch.where(c == 0, one * (1.0 - u * u), 0.5 * (u * u + c * u))
    if p == 1:
        return torch.where(c == 0, one * (-2.0 * u), u + 0.5 * c)
    return torch.where(c == 0, -one, 0.5 * one)


def unit_central_moment_dist(U, p):
    """Distribution with central moment 1 on cbar_x^px cbar_y^py cbar_z^pz and 0 on every other
    cbar monomial of degree <= 2 per axis: prod_a h_{p_a}(c_a; U_a). Returns (27, n)."""
    out = torch.ones((27,) + tuple(U[0].shape), dtype=U.dtype)
    for a in range(3):
        out = out * _h(p[a], C[:, a:a + 1], U[a])
    return out


def collide_closed(f, rho, U, B, omega, F=None):
    """Exact closed form of collide_T. f: (27, n)."""
    f0 = f_mhd_eq(rho, U, B)
    d = f - f0
    cb = C.T.unsqueeze(-1) - U.unsqueeze(1)                # (3, 27, n)
    K = torch.einsum("ain,bin,in->abn", cb, cb, d)         # second central moment of f - f0
    tr = (K[0, 0] + K[1, 1] + K[2, 2]) / 3.0
    P = K.clone()
    for a in range(3):
        P[a, a] = P[a, a] - tr
    out = f0.clone()
    pairs = {(0, 0): (2, 0, 0), (1, 1): (0, 2, 0), (2, 2): (0, 0, 2),
             (0, 1): (1, 1, 0), (0, 2): (1, 0, 1), (1, 2): (0, 1, 1)}
    for (a, b), p in pairs.items():
        out = out + (1.0 - omega) * P[a, b] * unit_central_moment_dist(U, p)
    if F is not None:
        for a, p in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            out = out + 0.5 * F[a] * unit_central_moment_dist(U, p)
    return out


def collide_bgk_closed(f, rho, U, B, omega, F=None):
    """Closed form of the BGK limit S = omega I of collide_T (Sec. 3.1.2: the BGK collision is
    the central-moment one with every rate equal to omega): f0 + (1 - omega)(f - f0). With a
    force the first central moments are set to F/2 as in the central-moment scheme; before the
    collision those of f - f0 are -F/2 (U carries F/2), so the force adds (1 - omega/2) F_a times
    the distribution with a unit first central moment along a."""
    f0 = f_mhd_eq(rho, U, B)
    out = f0 + (1.0 - omega) * (f - f0)
    if F is not None:
        for a, p in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            out = out + (1.0 - 0.5 * omega) * F[a] * unit_central_moment_dist(U, p)
    return out



def guo_force_dist(U, lat):
    """Second-order Hermite form of the distributions with a unit first central moment along
    each axis (and zero mass and second central moment), on a velocity set without the D3Q27
    corners: phi^a_i = w_i [(c_ia - U_a) / c_s^2 + (c_i . U) c_ia / c_s^4]. Returns (3, q, n)."""
    from .lattice import CS2
    c = lat.c.T.unsqueeze(-1)                                   # (3, q, 1)
    w = lat.w.view(1, -1, 1)
    cu = (c * U.unsqueeze(1)).sum(0, keepdim=True)             # (1, q, n)
    return w * ((c - U.unsqueeze(1)) / CS2 + cu * c / CS2 ** 2)


def collide_bgk_second_order(f, rho, U, B, omega, lat, F=None):
    """BGK collision (S = omega I, Sec. 3.1.1) on a fluid set without the D3Q27 corners, towards
    its second-order equilibrium with the Maxwell-stress term, f0 + (1 - omega)(f - f0); a body
    force adds (1 - omega/2) F_a phi^a (guo_force_dist), which, with U carrying F/(2 rho), ends
    the first central moments at +F/2 as in the D3Q27 operators. f: (q, n)."""
    from .equilibrium import f_mhd_eq_lattice
    f0 = f_mhd_eq_lattice(rho, U, B, lat)
    out = f0 + (1.0 - omega) * (f - f0)
    if F is not None:
        phi = guo_force_dist(U, lat)
        for a in range(3):
            out = out + (1.0 - 0.5 * omega) * F[a] * phi[a]
    return out
