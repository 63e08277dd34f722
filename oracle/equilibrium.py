"""Equilibria of the two schemes (paper Sec. 3.1, 3.2, App. A).

* f_eq: the sixth-order Hermite expansion of App. A, term by term. Two label misprints are
  read as the only index patterns that complete the fourth-order group: "H_xyyx" is
  H_xyyz (with U_x U_y^2 U_z), and "U_x^2 U_y U_y" is U_x^2 U_y U_z.
* maxwell_term: the Lorentz-force upgrade of the equilibrium. The printed term
  (w/2c_s^4)(|B|^2 |c|^2 - (c.B)^2) has mass 3|B|^2 and second moment 2|B|^2 I - BB,
  contradicting the moment the paper states it must produce (1/2 |B|^2 I - BB with
  unchanged mass and momentum). It is read as the Hermite projection of that stated
  moment: (w/2c_s^4) M : (c c - c_s^2 I) with M = 1/2 |B|^2 I - B B.
* g_eq_hall: the vector-valued D3Q7 equilibrium with the Hall correction U -> U - alpha_H J
  (eq. gHall_eq), also on the D3Q15 / D3Q27 magnetic variants.
* f_eq2: the second-order equilibrium of the D3Q19 fluid variant.

Shapes: scalars (...), vectors (3, ...), populations (27, ...) or (7, 3, ...).
"""

import torch

from .lattice import C, CS2, C2, W, WM, XI


def _bc(t, ref):
    """Broadcast a per-direction table (Q,) against fields of shape (...)."""
    return t.view(-1, *([1] * ref.dim()))


def hermite_polys(c, cs2=CS2):
    """Tensor Hermite polynomials of the velocity set, as a dict keyed by index string."""
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    ax, ay, az = cx * cx - cs2, cy * cy - cs2, cz * cz - cs2
    return {
        "xx": ax, "yy": ay, "zz": az, "xy": cx * cy, "xz": cx * cz, "yz": cy * cz,
        "xxy": ax * cy, "xxz": ax * cz, "xyy": cx * ay, "xzz": cx * az, "yzz": cy * az,
        "yyz": ay * cz, "xyz": cx * cy * cz,
        "xxyy": ax * ay, "xxzz": ax * az, "yyzz": ay * az,
        "xyzz": cx * cy * az, "xyyz": cx * ay * cz, "xxyz": ax * cy * cz,
        "xxyzz": ax * cy * az, "xxyyz": ax * ay * cz, "xyyzz": cx * ay * az,
        "xxyyzz": ax * ay * az,
    }


def f_eq(rho, U):
    """Sixth-order Hermite equilibrium f^(0)(rho, U) of App. A; returns (27, ...)."""
    H = {k: _bc(v, rho) for k, v in hermite_polys(C).items()}
    cs2 = CS2
    ux, uy, uz = U[0], U[1], U[2]
    cu = _bc(C[:, 0], rho) * ux + _bc(C[:, 1], rho) * uy + _bc(C[:, 2], rho) * uz
    o2 = (H["xx"] * ux * ux + H["yy"] * uy * uy + H["zz"] * uz * uz
          + 2.0 * (H["xy"] * ux * uy + H["xz"] * ux * uz + H["yz"] * uy * uz))
    o3 = (H["xxy"] * ux * ux * uy + H["xxz"] * ux * ux * uz + H["xyy"] * ux * uy * uy
          + H["xzz"] * ux * uz * uz + H["yzz"] * uy * uz * uz + H["yyz"] * uy * uy * uz
          + 2.0 * H["xyz"] * ux * uy * uz)
    o4 = (H["xxyy"] * ux * ux * uy * uy + H["xxzz"] * ux * ux * uz * uz
          + H["yyzz"] * uy * uy * uz * uz
          + 2.0 * (H["xyzz"] * ux * uy * uz * uz + H["xyyz"] * ux * uy * uy * uz
                   + H["xxyz"] * ux * ux * uy * uz))
    o5 = (H["xxyzz"] * ux * ux * uy * uz * uz + H["xxyyz"] * ux * ux * uy * uy * uz
          + H["xyyzz"] * ux * uy * uy * uz * uz)
    o6 = H["xxyyzz"] * ux * ux * uy * uy * uz * uz
    bracket = (1.0 + cu / cs2 + o2 / (2 * cs2 ** 2) + o3 / (2 * cs2 ** 3)
               + o4 / (4 * cs2 ** 4) + o5 / (4 * cs2 ** 5) + o6 / (8 * cs2 ** 6))
    return _bc(W, rho) * rho * bracket


def maxwell_term(B, c=C, w=W):
    """Lorentz-force part of the fluid equilibrium: (w/2c_s^4) M:(cc - c_s^2 I), on the velocity
    set c with weights w (the paper's D3Q27 by default)."""
    bx, by, bz = B[0], B[1], B[2]
    b2 = bx * bx + by * by + bz * bz
    M = [[0.5 * b2 - bx * bx, -bx * by, -bx * bz],
         [-by * bx, 0.5 * b2 - by * by, -by * bz],
         [-bz * bx, -bz * by, 0.5 * b2 - bz * bz]]
    out = torch.zeros((c.shape[0],) + tuple(bx.shape), dtype=bx.dtype)
    for a in range(3):
        for b in range(3):
            proj = _bc(c[:, a] * c[:, b] - (CS2 if a == b else 0.0), bx)
            out = out + proj * M[a][b]
    return _bc(w, bx) / (2 * CS2 ** 2) * out


def f_eq2(rho, U, c, w):
    """Second-order Hermite equilibrium on a velocity set without the D3Q27 corners (D3Q19):
    w rho (1 + c.U / c_s^2 + (c.U)^2 / (2 c_s^4) - |U|^2 / (2 c_s^2)), the truncation of the
    App. A expansion at the highest order whose Hermite polynomials such a set represents with
    the continuous-weight norms (its mass, momentum and momentum flux rho U U + rho c_s^2 I are
    exact)."""
    cu = _bc(c[:, 0], rho) * U[0] + _bc(c[:, 1], rho) * U[1] + _bc(c[:, 2], rho) * U[2]
    u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2]
    return _bc(w, rho) * rho * (1.0 + cu / CS2 + cu * cu / (2 * CS2 ** 2) - u2 / (2 * CS2))


def f_mhd_eq_lattice(rho, U, B, lat):
    """f^mhd(0)(rho, U, B) on the fluid lattice lat: the paper's sixth-order D3Q27 form, or the
    second-order form on D3Q19; both with the Maxwell-stress term."""
    if lat.name == "d3q27":
        return f_mhd_eq(rho, U, B)
    return f_eq2(rho, U, lat.c, lat.w) + maxwell_term(B, lat.c, lat.w)


def f_mhd_eq(rho, U, B):
    """f^mhd(0)(rho, U, B) = f^(0)(rho, U) + Maxwell-stress term."""
    return f_eq(rho, U) + maxwell_term(B)


def g_eq_hall(U, B, J, alpha_h, xi=XI, wm=WM):
    """Hall-MHD magnetic equilibrium, eq. gHall_eq; returns (M, 3, ...) on the magnetic velocity
    set xi with weights wm (the paper's D3Q7 by default).

    g_{i,a} = W_i (B_a + xi_{i,b} (V_b B_a - B_b V_a) / C^2) with V = U - alpha_H J.
    """
    V = U - alpha_h * J
    xv = torch.einsum("ib,b...->i...", xi, V)       # xi_i . V
    xb = torch.einsum("ib,b...->i...", xi, B)       # xi_i . B
    g = B.unsqueeze(0) + (xv.unsqueeze(1) * B.unsqueeze(0) - xb.unsqueeze(1) * V.unsqueeze(0)) / C2
    return wm.view(xi.shape[0], *([1] * B.dim())) * g
