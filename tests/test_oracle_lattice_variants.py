"""Pins of the lattice variants of the oracle (the D3Q19 fluid set; the D3Q15 and D3Q27 magnetic
sets of Sec. 4.3's closing remark): closed-form moment identities of the weights and equilibria,
conservation and the forcing budget of the second-order BGK collision, the exact Hall wave of
Sec. 4.1 with second-order convergence under diffusive scaling, the exact equivalence of the
magnetic sets for a field that varies along one axis only (the populations grouped by their
velocity component along that axis evolve as the D3Q7 ones), and the paper's statement that the
larger magnetic sets bring no significant gain in accuracy."""

import math

import numpy as np
import pytest
import torch

import synthetic
from oracle import analytic, collision, equilibrium, scheme
from oracle.lattice import C2, CS2, FLUID_LATTICES, MAGNETIC_LATTICES

DT = torch.float64


def _moment(lat, f, *axes):
    """sum_i f_i prod_a c_ia for f of shape (q, ...)."""
    w = torch.ones(lat.q, dtype=DT)
    for a in axes:
        w = w * lat.c[:, a]
    return torch.einsum("i,i...->...", w, f)


@pytest.mark.parametrize("name", ["d3q19", "d3q27"])
def test_fluid_weights(name):
    lat = FLUID_LATTICES[name]
    w, c = lat.w, lat.c
    assert abs(float(w.sum()) - 1.0) < 1e-15
    for a in range(3):
        assert abs(float((w * c[:, a]).sum())) < 1e-16
        for b in range(3):
            assert abs(float((w * c[:, a] * c[:, b]).sum()) - (CS2 if a == b else 0.0)) < 1e-16
    # fourth-order isotropy: sum w c_x^4 = 3 c_s^4, sum w c_x^2 c_y^2 = c_s^4
    assert abs(float((w * c[:, 0] ** 4).sum()) - 3 * CS2 ** 2) < 1e-16
    assert abs(float((w * c[:, 0] ** 2 * c[:, 1] ** 2).sum()) - CS2 ** 2) < 1e-16
    assert all(lat.opp[lat.opp[i]] == i for i in range(lat.q))
    if name == "d3q19":
        assert lat.q == 19 and all(int((c[i] ** 2).sum()) <= 2 for i in range(19))
        assert [lat.opp[i] for i in range(1, 10)] == list(range(10, 19))


@pytest.mark.parametrize("name", ["d3q7", "d3q15", "d3q27"])
def test_magnetic_weights(name):
    """sum W = 1 and sum W xi xi = C^2 I with C^2 = 1/4 (node coincidence, Sec. 3.2); the two
    larger sets are also isotropic at fourth order; each has the D3Q7 weights 1/8 along +-z after
    summing over the other two components (the grouping behind test_one_axis_equivalence)."""
    lat = MAGNETIC_LATTICES[name]
    w, c = lat.w, lat.c
    assert abs(float(w.sum()) - 1.0) < 1e-15
    for a in range(3):
        assert abs(float((w * c[:, a]).sum())) < 1e-16
        for b in range(3):
            assert abs(float((w * c[:, a] * c[:, b]).sum()) - (C2 if a == b else 0.0)) < 1e-16
    if name != "d3q7":
        assert abs(float((w * c[:, 0] ** 4).sum()) - 3 * float((w * c[:, 0] ** 2 * c[:, 1] ** 2).sum())) < 1e-16
        assert [lat.opp[i] for i in range(1, (lat.q + 1) // 2)] == list(range((lat.q + 1) // 2, lat.q))
    for s in (-1, 1):
        assert abs(float(w[c[:, 2] == s].sum()) - 0.125) < 1e-16


def test_d3q19_equilibrium_moments():
    """The second-order equilibrium reproduces mass, momentum and the momentum flux
    rho U U + rho c_s^2 I exactly; the Maxwell term adds M = |B|^2/2 I - B B to the flux and no
    mass or momentum."""
    lat = FLUID_LATTICES["d3q19"]
    g = torch.Generator().manual_seed(3)
    n = 50
    rho = 1.0 + 0.1 * torch.rand(n, generator=g, dtype=DT)
    U = 0.1 * torch.randn(3, n, generator=g, dtype=DT)
    B = 0.1 * torch.randn(3, n, generator=g, dtype=DT)
    f0 = equilibrium.f_eq2(rho, U, lat.c, lat.w)
    assert torch.allclose(_moment(lat, f0), rho, rtol=0, atol=1e-15)
    for a in range(3):
        assert torch.allclose(_moment(lat, f0, a), rho * U[a], rtol=0, atol=1e-16)
        for b in range(3):
            want = rho * U[a] * U[b] + (rho * CS2 if a == b else 0.0)
            assert torch.allclose(_moment(lat, f0, a, b), want, rtol=0, atol=1e-15)
    m = equilibrium.maxwell_term(B, lat.c, lat.w)
    b2 = (B * B).sum(0)
    assert float(_moment(lat, m).abs().max()) < 1e-16
    for a in range(3):
        assert float(_moment(lat, m, a).abs().max()) < 1e-16
        for b in range(3):
            want = (0.5 * b2 if a == b else 0.0) - B[a] * B[b]
            assert torch.allclose(_moment(lat, m, a, b), want, rtol=0, atol=1e-16)


@pytest.mark.parametrize("name", ["d3q15", "d3q27"])
def test_magnetic_equilibrium_moments(name):
    """sum_i g^Hall(0)_i = B, sum_i xi_ia g_ib = V_a B_b - B_a V_b (eq. Hall_eq_tensor) and
    sum_i xi_ia xi_ic g_ib = C^2 delta_ac B_b, with V = U - alpha_H J."""
    lat = MAGNETIC_LATTICES[name]
    g = torch.Generator().manual_seed(5)
    n = 40
    U, B, J = (0.1 * torch.randn(3, n, generator=g, dtype=DT) for _ in range(3))
    alpha = 1.7
    geq = equilibrium.g_eq_hall(U, B, J, alpha, lat.c, lat.w)      # (q, 3, n)
    V = U - alpha * J
    assert torch.allclose(geq.sum(0), B, rtol=0, atol=1e-15)
    for a in range(3):
        lam = torch.einsum("i,ibn->bn", lat.c[:, a], geq)
        assert torch.allclose(lam, V[a] * B - B[a] * V, rtol=0, atol=1e-15)
        for cc in range(3):
            second = torch.einsum("i,ibn->bn", lat.c[:, a] * lat.c[:, cc], geq)
            assert torch.allclose(second, (C2 * B) if a == cc else torch.zeros_like(B), rtol=0, atol=1e-15)


def test_guo_force_distribution_moments():
    """The second-order forcing distributions: zero mass, unit first central moment along their
    axis, zero second central moment."""
    lat = FLUID_LATTICES["d3q19"]
    g = torch.Generator().manual_seed(7)
    U = 0.1 * torch.randn(3, 30, generator=g, dtype=DT)
    phi = collision.guo_force_dist(U, lat)                          # (3, q, n)
    cb = lat.c.T.unsqueeze(-1) - U.unsqueeze(1)                     # (3, q, n)
    for a in range(3):
        assert float(phi[a].sum(0).abs().max()) < 1e-15
        for b in range(3):
            first = (phi[a] * cb[b]).sum(0)
            assert torch.allclose(first, torch.full_like(first, 1.0 if a == b else 0.0), rtol=0, atol=1e-15)
            for c in range(3):
                assert float((phi[a] * cb[b] * cb[c]).sum(0).abs().max()) < 1e-15


def test_d3q19_bgk_conservation_and_force():
    """The D3Q19 BGK collision conserves mass, adds F to the momentum (U carrying F/(2 rho)) and
    relaxes the non-equilibrium momentum flux at rate omega."""
    lat = FLUID_LATTICES["d3q19"]
    g = torch.Generator().manual_seed(9)
    n = 64
    rho0 = 1.0 + 0.05 * torch.rand(n, generator=g, dtype=DT)
    U0 = 0.05 * torch.randn(3, n, generator=g, dtype=DT)
    B = 0.05 * torch.randn(3, n, generator=g, dtype=DT)
    f = equilibrium.f_mhd_eq_lattice(rho0, U0, B, lat) + 1e-3 * torch.randn(19, n, generator=g, dtype=DT)
    F = 1e-3 * torch.randn(3, n, generator=g, dtype=DT)
    rho = f.sum(0)
    U = (torch.einsum("in,ia->an", f, lat.c) + 0.5 * F) / rho
    omega = 1.3
    fs = collision.collide_bgk_second_order(f, rho, U, B, omega, lat, F=F)
    assert torch.allclose(fs.sum(0), rho, rtol=0, atol=1e-15)
    mom = torch.einsum("in,ia->an", fs, lat.c)
    assert torch.allclose(mom, torch.einsum("in,ia->an", f, lat.c) + F, rtol=0, atol=1e-15)
    f0 = equilibrium.f_mhd_eq_lattice(rho, U, B, lat)
    for a, b in ((0, 0), (0, 1), (1, 2), (2, 2)):
        pre = _moment(lat, f - f0, a, b)
        post = _moment(lat, fs - f0, a, b)
        guo = (1 - 0.5 * omega) * (U[a] * F[b] + U[b] * F[a])
        assert torch.allclose(post, (1 - omega) * pre + guo, rtol=0, atol=1e-15)


def _wave(N, steps, amp, b0, d_i, fl, ml, branch=+1, jmode="moment", nx=1, ny=1):
    p = scheme.Params(nx, ny, N, 0.01, 0.01, d_i, (0.0, 0.0, b0), jmode, "closed",
                      collision="bgk" if fl == "d3q19" else "central", fluid_lattice=fl, magnetic_lattice=ml)
    be = analytic.beta(d_i, 2 * math.pi / N, branch)
    uf = synthetic.wave_field(amp)
    u, gu = synthetic.evaluate(uf, (nx, ny, N))
    b, gb = synthetic.evaluate(synthetic.scaled(uf, be), (nx, ny, N))
    return p, scheme.step(scheme.init_state(p, u, b, gu, gb), p, steps)


def _wave_error(N, steps, amp, b0, d_i, fl, ml, **kw):
    p, st = _wave(N, steps, amp, b0, d_i, fl, ml, **kw)
    _, U, B, _, _ = scheme.fields(st, p)
    ue, be = analytic.wave(N, steps, amp, b0, 0.01, d_i, kw.get("branch", +1))
    eu = torch.linalg.norm(U[:, :, 0, 0] - ue) / torch.linalg.norm(ue)
    bf = be.clone()
    bf[2] -= b0
    eb = torch.linalg.norm(B[:, :, 0, 0] - be) / torch.linalg.norm(bf)
    return float(eu), float(eb)


# Exact-wave bars (32 nodes per wavelength, 200 steps, beta+; as for the paper's lattices): the
# measured error times 1.25. Measured (u, b): D3Q19 fluid moment route 3.00% / 4.06%, stencil
# route 0.46% / 0.66%; the magnetic variants on D3Q27 fluid equal the D3Q7 values to 0.3%.
TOL_WAVE_VARIANT = {("d3q19", "moment"): 0.051, ("d3q19", "stencil"): 0.0083,
                    ("d3q27", "moment"): 0.051, ("d3q27", "stencil"): 0.0077}


@pytest.mark.parametrize("fl,ml", [("d3q19", "d3q7"), ("d3q27", "d3q15"), ("d3q27", "d3q27"), ("d3q19", "d3q15")])
@pytest.mark.parametrize("jmode", ["moment", "stencil"])
def test_variant_exact_wave_second_order(fl, ml, jmode):
    eu, eb = _wave_error(32, 200, 1e-3, 0.1, 2.0, fl, ml, jmode=jmode)
    tol = TOL_WAVE_VARIANT[(fl, jmode)]
    assert eu < tol and eb < tol, (eu, eb)
    Ns = [16, 32, 64]
    errs = []
    for N in Ns:
        s = N / 32
        errs.append(max(_wave_error(N, int(round(200 * s * s)), 1e-3 / s, 0.1 / s, 2.0 * s, fl, ml, jmode=jmode)))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert slope < -1.8, (errs, slope)


def test_one_axis_equivalence_of_magnetic_sets():
    """For fields that vary along z only, the magnetic populations grouped by xi_z evolve exactly
    as the D3Q7 ones (each group carries the weight 1/8 along +-z, the equilibrium's transverse
    terms cancel within a group, and streaming moves a whole group along z): with J from the
    curl of B, B of the D3Q15 and D3Q27 runs equals that of the D3Q7 run to rounding. A wrong
    weight in either larger set breaks this."""
    ref = None
    for ml in ("d3q7", "d3q15", "d3q27"):
        p, st = _wave(32, 150, 1e-3, 0.1, 2.0, "d3q27", ml, jmode="stencil")
        B = st.g.sum(0)
        grouped = torch.stack([st.g[p.ml.c[:, 2] == s].sum(0) for s in (-1, 0, 1)])
        if ref is None:
            ref = (B, grouped)
            continue
        # rounding of sums of O(0.1) values over 150 steps; a wrong weight shows at the 1e-4 level
        assert float((B - ref[0]).abs().max()) < 1e-14
        assert float((grouped - ref[1]).abs().max()) < 1e-14


def test_larger_magnetic_sets_bring_no_significant_gain():
    """Sec. 4.3: upgrading the magnetic lattice from D3Q7 to D3Q15 or D3Q27 does not improve the
    accuracy significantly. On the exact Hall wave with J from the magnetic moments (the paper's
    route) the errors of the three sets agree to 1% of their size on both branches."""
    for branch in (+1, -1):
        e7 = _wave_error(32, 200, 1e-3, 0.1, 2.0, "d3q27", "d3q7", branch=branch)
        for ml in ("d3q15", "d3q27"):
            e = _wave_error(32, 200, 1e-3, 0.1, 2.0, "d3q27", ml, branch=branch)
            for x, y in zip(e, e7):
                assert abs(x - y) < 0.01 * y, (ml, branch, e, e7)


@pytest.mark.parametrize("fl,ml", [("d3q19", "d3q7"), ("d3q27", "d3q15"), ("d3q19", "d3q27")])
def test_variant_invariants(fl, ml):
    """Mass, momentum (+F per step) and the summed field (+S per step) are exact invariants of the
    variant steps too, on a forced turbulent 8^3 state."""
    n = 8
    shape = (n, n, n)
    u, gu = synthetic.evaluate(synthetic.shell_field(0, 1, 2, 0.02), shape)
    b, gb = synthetic.evaluate(synthetic.shell_field(1, 1, 2, 0.02), shape)
    fu, _ = synthetic.evaluate(synthetic.shell_field(2, 0, 2, 1e-4, "radius"), shape, gradient=False)
    fb, _ = synthetic.evaluate(synthetic.shell_field(3, 0, 2, 1e-4, "radius"), shape, gradient=False)
    fu = fu + torch.tensor([2e-5, -1e-5, 3e-5], dtype=DT).view(3, 1, 1, 1)
    fb = fb + torch.tensor([-1e-5, 2e-5, 1e-5], dtype=DT).view(3, 1, 1, 1)
    p = scheme.Params(n, n, n, 0.02, 0.03, 2.0, (0.01, -0.02, 0.05), "moment", "closed", fu, fb,
                      collision="bgk" if fl == "d3q19" else "central", fluid_lattice=fl, magnetic_lattice=ml)
    st = scheme.init_state(p, u, b, gu, gb)
    mass0 = float(st.f.sum())
    mom0 = torch.einsum("i...,ia->a", st.f, p.fl.c)
    bsum0 = st.g.sum((0, 2, 3, 4))
    steps = 7
    st = scheme.step(st, p, steps)
    assert abs(float(st.f.sum()) - mass0) < 1e-12 * mass0
    mom = torch.einsum("i...,ia->a", st.f, p.fl.c)
    assert torch.allclose(mom - mom0, steps * fu.sum((1, 2, 3)), rtol=1e-12, atol=1e-13)
    assert torch.allclose(st.g.sum((0, 2, 3, 4)) - bsum0, steps * fb.sum((1, 2, 3)), rtol=1e-12, atol=1e-13)


def test_initial_state_moments_d3q19():
    """The D3Q19 initial state returns rho = 1, u and B = b0 + b, and its deviatoric momentum
    flux departs from equilibrium by -(c_s^2 / omega)(grad u + grad u^T - 2/3 div u I)."""
    n = 6
    shape = (n, n, n)
    u, gu = synthetic.evaluate(synthetic.shell_field(4, 1, 2, 0.02), shape)
    b, gb = synthetic.evaluate(synthetic.shell_field(5, 1, 2, 0.02), shape)
    p = scheme.Params(n, n, n, 0.02, 0.03, 2.0, (0.01, -0.02, 0.05), "moment", "closed", collision="bgk",
                      fluid_lattice="d3q19", magnetic_lattice="d3q15")
    st = scheme.init_state(p, u, b, gu, gb)
    rho, U, B, _ = scheme.moments(st, p)
    assert float((rho - 1).abs().max()) < 1e-15
    assert float((U - u).abs().max()) < 1e-16
    assert float((B - b - torch.tensor(p.b0, dtype=DT).view(3, 1, 1, 1)).abs().max()) < 1e-16
    lat = p.fl
    f0 = equilibrium.f_mhd_eq_lattice(rho, U, B, lat)
    for a, c in ((0, 1), (1, 2), (0, 0)):
        got = _moment(lat, st.f - f0, a, c)
        s = gu[a, c] + gu[c, a]
        want = -(CS2 / p.omega) * (s - ((2.0 / 3.0) * (gu[0, 0] + gu[1, 1] + gu[2, 2]) if a == c else 0.0))
        assert torch.allclose(got, want, rtol=0, atol=1e-15)
