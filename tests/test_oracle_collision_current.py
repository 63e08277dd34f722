"""Pins of the oracle's fluid collision (Sec. 3.1.2, App. A) and current density (Sec. 3.2,
App. B) against invariants, special cases and the paper's printed closed forms.
"""

import itertools
import math

import torch

from oracle import collision as col
from oracle import current as cur
from oracle.equilibrium import f_mhd_eq
from oracle.lattice import C, C2

torch.manual_seed(1)


def _random_populations(n, amp=0.02):
    rho = 1.0 + 0.05 * torch.randn(n, dtype=torch.float64)
    U = 0.08 * torch.randn(3, n, dtype=torch.float64)
    B = 0.1 * torch.randn(3, n, dtype=torch.float64)
    f = f_mhd_eq(rho, U, B) + amp * torch.randn(27, n, dtype=torch.float64) / 27
    rho = f.sum(0)
    U = torch.einsum("in,ia->an", f, C) / rho
    return f, rho, U, B


def test_printed_basis_is_singular_and_corrected_basis_is_not():
    U = 0.05 * torch.randn(3, 6, dtype=torch.float64)
    assert int(torch.linalg.matrix_rank(col.t_matrix(U, printed=True)[0])) == 26
    assert all(int(torch.linalg.matrix_rank(t)) == 27 for t in col.t_matrix(U))


def test_collision_conserves_mass_and_momentum():
    f, rho, U, B = _random_populations(300)
    fs = col.collide_T(f, rho, U, B, omega=1.7)
    assert torch.allclose(fs.sum(0), rho, atol=1e-14, rtol=0)
    assert torch.allclose(torch.einsum("in,ia->an", fs, C), rho * U, atol=1e-15, rtol=0)


def test_T_route_equals_closed_form():
    f, rho, U, B = _random_populations(500)
    F = 1e-3 * torch.randn(3, 500, dtype=torch.float64)
    for omega in (0.6, 1.0, 1.9):
        a = col.collide_T(f, rho, U, B, omega)
        b = col.collide_closed(f, rho, U, B, omega)
        assert (a - b).abs().max() < 1e-15
        a = col.collide_T(f, rho, U, B, omega, F=F)
        b = col.collide_closed(f, rho, U, B, omega, F=F)
        assert (a - b).abs().max() < 1e-15


def test_bgk_limit():
    # S = omega I reproduces the BGK collision f - omega (f - f0) (Sec. 3.1.2)
    f, rho, U, B = _random_populations(200)
    omega = 1.3
    fs = col.collide_T(f, rho, U, B, omega, rates=torch.full((27,), omega, dtype=torch.float64))
    assert (fs - (f - omega * (f - f_mhd_eq(rho, U, B)))).abs().max() < 1e-15


def test_bgk_closed_form_equals_T_route():
    """The BGK variant's closed form against the definition with every rate equal to omega, with
    and without a force (first central moments set to F/2); the force adds F to the momentum."""
    f, rho, U0, B = _random_populations(300)
    F = 1e-3 * torch.randn(3, 300, dtype=torch.float64)
    mom = torch.einsum("in,ia->an", f, C)
    U = (mom + 0.5 * F) / rho
    for omega in (0.6, 1.0, 1.9):
        rates = torch.full((27,), omega, dtype=torch.float64)
        for FF, UU in ((None, U0), (F, U)):
            a = col.collide_T(f, rho, UU, B, omega, F=FF, rates=rates)
            b = col.collide_bgk_closed(f, rho, UU, B, omega, F=FF)
            assert (a - b).abs().max() < 1e-15
        fs = col.collide_bgk_closed(f, rho, U, B, omega, F=F)
        assert torch.allclose(torch.einsum("in,ia->an", fs, C), mom + F, atol=1e-15, rtol=0)
        assert torch.allclose(fs.sum(0), rho, atol=1e-14, rtol=0)


def test_post_collision_central_moments():
    # second-order deviatoric non-equilibrium scaled by (1 - omega); trace and every
    # higher moment (per-axis degree <= 2) at equilibrium
    f, rho, U, B = _random_populations(100)
    omega = 1.45
    f0 = f_mhd_eq(rho, U, B)
    fs = col.collide_T(f, rho, U, B, omega)
    cb = C.unsqueeze(-1) - U.unsqueeze(0)
    def cm(g, p):
        return (g * cb[:, 0] ** p[0] * cb[:, 1] ** p[1] * cb[:, 2] ** p[2]).sum(0)
    for p in itertools.product(range(3), repeat=3):
        d_post = cm(fs - f0, p)
        if sum(p) == 2 and max(p) == 1:              # off-diagonal second moments
            assert torch.allclose(d_post, (1 - omega) * cm(f - f0, p), atol=1e-15)
        elif sum(p) >= 3 or sum(p) <= 1:
            assert d_post.abs().max() < 1e-15, p
    tr_post = sum(cm(fs - f0, p) for p in [(2, 0, 0), (0, 2, 0), (0, 0, 2)])
    assert tr_post.abs().max() < 1e-15
    dxx = cm(fs - f0, (2, 0, 0)) - cm(fs - f0, (0, 2, 0))
    assert torch.allclose(dxx, (1 - omega) * (cm(f - f0, (2, 0, 0)) - cm(f - f0, (0, 2, 0))), atol=1e-15)


def test_collision_independent_of_higher_order_basis():
    # another invertible basis that keeps T_0..T_9 and spans the higher monomials differently
    # (plain monomials) gives the same post-collision populations
    f, rho, U, B = _random_populations(100)
    omega = 1.2
    f0 = f_mhd_eq(rho, U, B)
    cb = C.unsqueeze(0) - U.T.unsqueeze(1)
    T = col.t_matrix(U)
    x, y, z = cb[..., 0], cb[..., 1], cb[..., 2]
    hi = [x * y * y, x * z * z, x * x * y, y * z * z, x * x * z, y * y * z, x * y * z,
          x * x * y * y, x * x * z * z, y * y * z * z, x * x * y * z, x * y * y * z, x * y * z * z,
          x * y * y * z * z, x * x * y * z * z, x * x * y * y * z, x * x * y * y * z * z]
    T2 = torch.cat([T[..., :10], torch.stack(hi, -1)], dim=-1)
    s = col.relaxation_rates(omega)
    dk = torch.einsum("mij,im->mj", T2, f - f0)
    sol = torch.linalg.solve(T2.transpose(1, 2), ((1 - s) * dk).unsqueeze(-1)).squeeze(-1).T
    assert (f0 + sol - col.collide_T(f, rho, U, B, omega)).abs().max() < 1e-15


def test_forcing_adds_F_to_momentum():
    f, rho, U0, B = _random_populations(100)
    F = 1e-3 * torch.randn(3, 100, dtype=torch.float64)
    mom = torch.einsum("in,ia->an", f, C)
    U = (mom + 0.5 * F) / rho
    fs = col.collide_T(f, rho, U, B, 1.5, F=F)
    assert torch.allclose(torch.einsum("in,ia->an", fs, C), mom + F, atol=1e-15, rtol=0)
    assert torch.allclose(fs.sum(0), rho, atol=1e-14, rtol=0)


# ---------------------------------------------------------------- current density

def test_moment_current_self_consistent():
    n = 50
    U = 0.05 * torch.randn(3, n, dtype=torch.float64)
    B = 0.2 * torch.randn(3, n, dtype=torch.float64)
    Lam = 0.01 * torch.randn(3, 3, n, dtype=torch.float64)
    for alpha in (0.0, 2.0, 16.0):
        omega_b = 1.9
        J = cur.current_moment(Lam, U, B, alpha, omega_b)
        V = U - alpha * J
        lam0 = torch.einsum("an,bn->abn", V, B) - torch.einsum("an,bn->abn", B, V)
        # eq. LB_density_current: J_g = -eps_abg (w_B / C^2)(Lambda_ab - Lambda0_ab)
        rhs = -(omega_b / C2) * cur.levi_civita_contract(Lam - lam0)
        assert (J - rhs).abs().max() < 1e-14 * max(1.0, J.abs().max().item())


def test_moment_current_ideal_limit():
    n = 20
    U = 0.05 * torch.randn(3, n, dtype=torch.float64)
    B = 0.2 * torch.randn(3, n, dtype=torch.float64)
    Lam = 0.01 * torch.randn(3, 3, n, dtype=torch.float64)
    J = cur.current_moment(Lam, U, B, 0.0, 1.5)
    assert torch.allclose(J, -(1.5 / C2) * cur.j0_vector(Lam, U, B), atol=1e-16)


def _app_b(Lam, U, B, aH, wB, c2=C2, fix=True):
    """App. B explicit solution, transcribed term by term. With fix=False the two printed
    terms read as misprints are kept: J_y's "+2 C^4 w_B B_z U_x" and J_z's "Lambda_zy B_x B_y"."""
    C4, C6 = c2 * c2, c2 ** 3
    Bx, By, Bz = B
    Ux, Uy, Uz = U
    L = lambda a, b: Lam["xyz".index(a), "xyz".index(b)]  # noqa: E731
    k1, k2, k3 = C4 * wB, c2 * aH * wB ** 2, aH ** 2 * wB ** 3
    D = C6 + 4 * c2 * aH ** 2 * wB ** 2 * (Bx * Bx + By * By + Bz * Bz)
    jx = (-2 * k1 * By * Uz + 2 * k1 * Bz * Uy - k1 * L("y", "z") + k1 * L("z", "y")
          - 4 * k2 * Bx * By * Uy - 4 * k2 * Bx * Bz * Uz + 4 * k2 * By ** 2 * Ux
          - 2 * k2 * L("x", "y") * By + 2 * k2 * L("y", "x") * By + 4 * k2 * Bz ** 2 * Ux
          - 2 * k2 * L("x", "z") * Bz + 2 * k2 * L("z", "x") * Bz - 4 * k3 * L("y", "z") * Bx ** 2
          + 4 * k3 * L("z", "y") * Bx ** 2 + 4 * k3 * L("x", "z") * Bx * By
          - 4 * k3 * L("z", "x") * Bx * By - 4 * k3 * L("x", "y") * Bx * Bz
          + 4 * k3 * L("y", "x") * Bx * Bz) / D
    s = -1.0 if fix else 1.0
    jy = (2 * k1 * Bx * Uz + s * 2 * k1 * Bz * Ux + k1 * L("x", "z") - k1 * L("z", "x")
          + 4 * k2 * Bx ** 2 * Uy - 4 * k2 * Bx * By * Ux + 2 * k2 * L("x", "y") * Bx
          - 2 * k2 * L("y", "x") * Bx - 4 * k2 * By * Bz * Uz + 4 * k2 * Bz ** 2 * Uy
          - 2 * k2 * L("y", "z") * Bz + 2 * k2 * L("z", "y") * Bz - 4 * k3 * L("y", "z") * Bx * By
          + 4 * k3 * L("z", "y") * Bx * By + 4 * k3 * L("x", "z") * By ** 2
          - 4 * k3 * L("z", "x") * By ** 2 - 4 * k3 * L("x", "y") * By * Bz
          + 4 * k3 * L("y", "x") * By * Bz) / D
    last = Bz if fix else By
    jz = (-2 * k1 * Bx * Uy + 2 * k1 * By * Ux - k1 * L("x", "y") + k1 * L("y", "x")
          + 4 * k2 * Bx ** 2 * Uz - 4 * k2 * Bx * Bz * Ux + 2 * k2 * L("x", "z") * Bx
          - 2 * k2 * L("z", "x") * Bx + 4 * k2 * By ** 2 * Uz - 4 * k2 * By * Bz * Uy
          + 2 * k2 * L("y", "z") * By - 2 * k2 * L("z", "y") * By - 4 * k3 * L("y", "z") * Bx * Bz
          + 4 * k3 * L("z", "y") * Bx * last + 4 * k3 * L("x", "z") * By * Bz
          - 4 * k3 * L("z", "x") * By * Bz - 4 * k3 * L("x", "y") * Bz ** 2
          + 4 * k3 * L("y", "x") * Bz ** 2) / D
    return torch.stack([jx, jy, jz])


def test_moment_current_matches_appendix_b():
    n = 64
    U = 0.05 * torch.randn(3, n, dtype=torch.float64)
    B = 0.3 * torch.randn(3, n, dtype=torch.float64)
    Lam = 0.02 * torch.randn(3, 3, n, dtype=torch.float64)
    aH, wB = 4.0, 1.8
    J = cur.current_moment(Lam, U, B, aH, wB)
    assert (J - _app_b(Lam, U, B, aH, wB)).abs().max() < 1e-14
    printed = _app_b(Lam, U, B, aH, wB, fix=False)
    assert (J[0] - printed[0]).abs().max() < 1e-14           # J_x is printed correctly
    assert (J[1] - printed[1]).abs().max() > 1e-6            # J_y, J_z carry a misprint each
    assert (J[2] - printed[2]).abs().max() > 1e-6


def test_stencil_current_single_mode():
    # central-difference curl of a Fourier mode = (sin k / k) x exact curl
    n = 16
    m = 3
    k = 2 * math.pi * m / n
    y = torch.arange(n, dtype=torch.float64).view(1, n, 1)
    B = torch.zeros(3, n, n, n, dtype=torch.float64)
    B[2] = torch.sin(k * y).expand(n, n, n)      # B_z(y): curl = (dBz/dy, 0, 0)
    B[0] = torch.cos(k * y).expand(n, n, n)      # B_x(y): curl_z = -dBx/dy
    J = cur.current_stencil(B)
    exact_x = k * torch.cos(k * y).expand(n, n, n)
    exact_z = k * torch.sin(k * y).expand(n, n, n)
    s = math.sin(k) / k
    assert (J[0] - s * exact_x).abs().max() < 1e-14
    assert (J[2] - s * exact_z).abs().max() < 1e-14
    assert J[1].abs().max() < 1e-15


def test_divergence_estimate_of_trace():
    Lam = torch.randn(3, 3, 5, dtype=torch.float64)
    d = cur.divergence_moment(Lam, 1.6)
    assert torch.allclose(d, -(1.6 / C2) * (Lam[0, 0] + Lam[1, 1] + Lam[2, 2]))


def test_central_gradient_single_modes():
    # central difference of a Fourier mode along each axis = (sin k / k) x exact derivative,
    # with the derivative direction first: grad[a, b] = d_a v_b
    from oracle import scheme
    n = 12
    x = torch.arange(n, dtype=torch.float64)
    v = torch.zeros(3, n, n, n, dtype=torch.float64)
    ks = {}
    for b, (axis, m) in enumerate(((0, 1), (1, 2), (2, 5))):     # v_b varies along axis b only
        k = 2 * math.pi * m / n
        shape = [1, 1, 1]
        shape[2 - axis] = n                                          # (z, y, x) tensor dims
        v[b] = torch.sin(k * x.view(shape)).expand(n, n, n)
        ks[b] = (axis, k, shape)
    g = scheme.central_gradient(v)
    for b, (axis, k, shape) in ks.items():
        exact = k * torch.cos(k * x.view(shape)).expand(n, n, n)
        assert (g[axis, b] - math.sin(k) / k * exact).abs().max() < 1e-14
        for a in range(3):
            if a != axis:
                assert g[a, b].abs().max() == 0.0
