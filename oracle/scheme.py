"""One time step of the coupled Hall-MHD lattice-Boltzmann scheme (paper Sec. 3), initial
state, and node fields.

Per node x, with lattice units dx = dt = 1:
 1. moments: rho = sum f, rho U = sum f c (+ F/2), B = sum g (+ S/2),
    Lambda_ab = sum_i xi_ia g_ib (eqs. LB_moments2, mag_field_LB, LB_density_current);
 2. J from the moments (3x3 solve) or from the central-difference curl of B;
 3. fluid: central-moment collision towards f^mhd(0)(rho, U, B) (eq. cm_collision_step);
 4. magnetic: BGK towards g^Hall(0)(U, B, J) (eq. MHD_LBscheme)
    [+ (1 - w_B/2) W_i S with a magnetic source S];
 5. stream both sets along their velocities, periodic (eq. stream).

State layout: f (27, nz, ny, nx), g (7, 3, nz, ny, nx), post-streaming / pre-collision,
velocity order as in oracle.lattice.

Initial state (the paper only fixes rho = 1): f = f^mhd(0)(1, u, B) plus the first-order
non-equilibrium part whose deviatoric second central moment is
-(rho c_s^2 / w)(grad u + grad u^T - 2/3 div u I); g = g^Hall(0)(u, B, curl B) plus
-(1 / w_B) W_i xi_ia d_a B_b, so that Lambda - Lambda0 = -(C^2 / w_B) grad B at t = 0.
With forcing, -F/2 and -S/2 are added so that the node moments return exactly u and B.

Variants (Params.collision, Params.magnetic): the BGK fluid collision, which is the same step
with S = omega I (Sec. 3.1.2); and electron MHD (Sec. 6), whose magnetic equilibrium, the J
system built on it and the initial magnetic state take the bulk velocity as zero.

Lattice variants (Params.fluid_lattice, Params.magnetic_lattice; readings in oracle.lattice):
the D3Q19 fluid set, which carries the BGK collision towards its second-order equilibrium with
the Maxwell-stress term (the central-moment operator of Sec. 3.1.2 is built on the 27-moment
basis of D3Q27), and the D3Q15 / D3Q27 magnetic sets, with the same Hall equilibrium and BGK
collision as D3Q7. The state then holds (q, ...) fluid and (m, 3, ...) magnetic populations.
For D3Q19 the initial non-equilibrium part is the second-order Hermite projection
(w / 2 c_s^4) P:(c c - c_s^2 I) of the same deviatoric moment P, and the forcing shift
-F/2 of the first central moments uses the second-order form of oracle.collision.guo_force_dist.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import collision
from .current import current_moment, current_stencil, divergence_moment
from .equilibrium import f_mhd_eq_lattice, g_eq_hall
from .lattice import CS2, DT, FLUID_LATTICES, MAGNETIC_LATTICES, omega_fluid, omega_magnetic


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    nz: int
    nu: float
    eta: float
    d_i: float = 0.0                       # Hall coefficient alpha_H in lattice units (rho0 = 1)
    b0: tuple = (0.0, 0.0, 0.0)            # uniform background field
    jmode: str = "moment"                  # "moment" (paper) or "stencil"
    route: str = "T"                       # fluid collision: "T" (definition) or "closed"
    force_u: Optional[torch.Tensor] = None  # (3, nz, ny, nx) fluid body force F
    force_b: Optional[torch.Tensor] = None  # (3, nz, ny, nx) magnetic source S
    # fluid collision: "central" (the paper's central-moment MRT, eq. collision_matrix) or "bgk"
    # (S = omega I, the standard BGK operator of Sec. 3.1.1)
    collision: str = "central"
    # magnetic equilibrium: "hall" (eq. gHall_eq, V = U - alpha_H J) or "emhd" (electron MHD,
    # Sec. 6: the bulk velocity neglected against the Hall current, V = -alpha_H J)
    magnetic: str = "hall"
    # velocity sets: the paper's D3Q27 fluid and D3Q7 magnetic, or the variants of oracle.lattice
    fluid_lattice: str = "d3q27"
    magnetic_lattice: str = "d3q7"

    @property
    def fl(self):
        return FLUID_LATTICES[self.fluid_lattice]

    @property
    def ml(self):
        return MAGNETIC_LATTICES[self.magnetic_lattice]

    @property
    def omega(self):
        return omega_fluid(self.nu)

    @property
    def omega_b(self):
        return omega_magnetic(self.eta)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class State:
    f: torch.Tensor   # (27, nz, ny, nx); (q, ...) on a fluid variant
    g: torch.Tensor   # (7, 3, nz, ny, nx); (m, 3, ...) on a magnetic variant

    def clone(self):
        return State(self.f.clone(), self.g.clone())


def moments(st: State, p: Params):
    """rho (nz,ny,nx), U (3,...), B (3,...), Lambda (3,3,...)."""
    rho = st.f.sum(0)
    mom = torch.einsum("i...,ia->a...", st.f, p.fl.c)
    if p.force_u is not None:
        mom = mom + 0.5 * p.force_u
    U = mom / rho
    B = st.g.sum(0)
    if p.force_b is not None:
        B = B + 0.5 * p.force_b
    Lam = torch.einsum("ia,ib...->ab...", p.ml.c, st.g)
    return rho, U, B, Lam


def magnetic_velocity(p: Params, U):
    """The bulk velocity as the magnetic equilibrium and the J system see it: U, or 0 for
    electron MHD."""
    if p.magnetic == "hall":
        return U
    if p.magnetic == "emhd":
        return torch.zeros_like(U)
    raise ValueError(p.magnetic)


def current(p: Params, U, B, Lam):
    """J of the current route; U is the magnetic_velocity."""
    if p.jmode == "moment":
        sh = B.shape[1:]
        n = B[0].numel()
        J = current_moment(Lam.reshape(3, 3, n), U.reshape(3, n), B.reshape(3, n), p.d_i, p.omega_b)
        return J.reshape((3,) + tuple(sh))
    if p.jmode == "stencil":
        return current_stencil(B)
    raise ValueError(p.jmode)


def collide(st: State, p: Params) -> State:
    """Post-collision populations at every node."""
    rho, U, B, Lam = moments(st, p)
    Um = magnetic_velocity(p, U)
    J = current(p, Um, B, Lam)
    n = p.ncell
    F = None if p.force_u is None else p.force_u.reshape(3, n)
    q = p.fl.q
    args = (st.f.reshape(q, n), rho.reshape(n), U.reshape(3, n), B.reshape(3, n), p.omega)
    if p.collision not in ("central", "bgk"):
        raise ValueError(p.collision)
    if p.fluid_lattice != "d3q27":
        if p.collision != "bgk":
            raise ValueError("the central-moment collision is defined on D3Q27 only")
        fs = collision.collide_bgk_second_order(*args, p.fl, F=F)
    elif p.route == "T":
        rates = torch.full((27,), p.omega, dtype=DT) if p.collision == "bgk" else None
        fs = collision.collide_T(*args, F=F, rates=rates)
    elif p.route == "closed":
        fs = (collision.collide_bgk_closed if p.collision == "bgk" else collision.collide_closed)(*args, F=F)
    else:
        raise ValueError(p.route)
    ml = p.ml
    geq = g_eq_hall(Um, B, J, p.d_i, ml.c, ml.w)
    gs = st.g - p.omega_b * (st.g - geq)
    if p.force_b is not None:
        gs = gs + (1.0 - 0.5 * p.omega_b) * ml.w.view(ml.q, 1, 1, 1, 1) * p.force_b.unsqueeze(0)
    return State(fs.reshape(st.f.shape), gs)


def stream(st: State, p: Optional[Params] = None) -> State:
    """f_i(x + c_i) <- f*_i(x); g_i(x + xi_i) <- g*_i(x), periodic (on the lattices of p; the
    paper's D3Q27 / D3Q7 without p)."""
    fc = FLUID_LATTICES["d3q27"].c if p is None else p.fl.c
    mc = MAGNETIC_LATTICES["d3q7"].c if p is None else p.ml.c
    f = torch.stack([torch.roll(st.f[i], shifts=(int(fc[i, 2]), int(fc[i, 1]), int(fc[i, 0])),
                                dims=(0, 1, 2)) for i in range(fc.shape[0])])
    g = torch.stack([torch.roll(st.g[i], shifts=(int(mc[i, 2]), int(mc[i, 1]), int(mc[i, 0])),
                                dims=(1, 2, 3)) for i in range(mc.shape[0])])
    return State(f, g)


def step(st: State, p: Params, nsteps: int = 1) -> State:
    for _ in range(nsteps):
        st = stream(collide(st, p), p)
    return st


def central_gradient(v):
    """grad[a, b] = (v_b(x + e_a) - v_b(x - e_a)) / 2 on the periodic grid, v of shape
    (3, nz, ny, nx): the second-order central difference that stands in for exact gradients
    at initialisation when none are given (the same stencil as the curl route of J)."""
    axis = {0: 3, 1: 2, 2: 1}          # tensor dimension of x, y, z
    return torch.stack([0.5 * (torch.roll(v, -1, dims=axis[a]) - torch.roll(v, 1, dims=axis[a]))
                        for a in range(3)])


def curl_from_gradient(grad):
    """(curl B)_g from grad[a, b] = d_a B_b."""
    return torch.stack([grad[1, 2] - grad[2, 1], grad[2, 0] - grad[0, 2], grad[0, 1] - grad[1, 0]])


def init_state(p: Params, u, b, grad_u=None, grad_b=None, noneq=True) -> State:
    """Initial populations from velocity u and field fluctuation b (B = b0 + b), rho = 1.

    grad_u[a, b] = d_a u_b and grad_b[a, b] = d_a b_b (exact gradients); they are needed for
    the non-equilibrium parts and for J = curl B in the Hall equilibrium.
    """
    n = p.ncell
    sh = p.shape
    fl, ml = p.fl, p.ml
    b0 = torch.tensor(p.b0, dtype=DT).view(3, 1, 1, 1)
    B = b + b0
    rho = torch.ones(sh, dtype=DT)
    f = f_mhd_eq_lattice(rho, u, B, fl)
    J = torch.zeros_like(u) if grad_b is None else curl_from_gradient(grad_b)
    g = g_eq_hall(magnetic_velocity(p, u), B, J, p.d_i, ml.c, ml.w)
    P = None
    if noneq and grad_u is not None:
        s = grad_u + grad_u.transpose(0, 1)
        div = grad_u[0, 0] + grad_u[1, 1] + grad_u[2, 2]
        P = -(CS2 / p.omega) * s
        for a in range(3):
            P[a, a] = P[a, a] + (CS2 / p.omega) * (2.0 / 3.0) * div
        P = P.reshape(3, 3, n)
    if fl.name == "d3q27":
        kneq = torch.zeros((n, 27), dtype=DT)
        if P is not None:
            kneq[:, 4], kneq[:, 5], kneq[:, 6] = P[0, 1], P[0, 2], P[1, 2]
            kneq[:, 7], kneq[:, 8] = P[0, 0] - P[1, 1], P[0, 0] - P[2, 2]
        if p.force_u is not None:
            kneq[:, 1:4] = -0.5 * p.force_u.reshape(3, n).T
        if bool(torch.any(kneq != 0)):
            f = f + collision.moments_to_dist(u.reshape(3, n), kneq).reshape((27,) + sh)
    else:
        # second-order Hermite projections of the same non-equilibrium moments
        fq = f.reshape(fl.q, n)
        if P is not None:
            for a in range(3):
                for bb in range(3):
                    proj = (fl.c[:, a] * fl.c[:, bb] - (CS2 if a == bb else 0.0)).view(-1, 1)
                    fq = fq + fl.w.view(-1, 1) / (2 * CS2 ** 2) * proj * P[a, bb].view(1, n)
        if p.force_u is not None:
            phi = collision.guo_force_dist(u.reshape(3, n), fl)
            F = p.force_u.reshape(3, n)
            for a in range(3):
                fq = fq - 0.5 * F[a] * phi[a]
        f = fq.reshape((fl.q,) + sh)
    if noneq and grad_b is not None:
        for i in range(ml.q):
            for bb in range(3):
                s = sum(ml.c[i, a] * grad_b[a, bb] for a in range(3) if ml.c[i, a] != 0)
                if not isinstance(s, int):
                    g[i, bb] = g[i, bb] - (1.0 / p.omega_b) * ml.w[i] * s
    if p.force_b is not None:
        g = g - 0.5 * ml.w.view(ml.q, 1, 1, 1, 1) * p.force_b.unsqueeze(0)
    return State(f, g)


def fields(st: State, p: Params):
    """Node fields of the current state: rho, u, B, J, div B (moment estimate)."""
    rho, U, B, Lam = moments(st, p)
    J = current(p, magnetic_velocity(p, U), B, Lam)
    return rho, U, B, J, divergence_moment(Lam, p.omega_b)


def rest_state(p: Params) -> State:
    """f^mhd(0)(1, 0, b0), g = W_i b0: the uniform state deviations are measured from."""
    sh = p.shape
    z = torch.zeros((3,) + sh, dtype=DT)
    return init_state(dataclasses.replace(p, force_u=None, force_b=None), z, z, noneq=False)
