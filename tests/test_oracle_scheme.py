"""Pins of the whole oracle step against the exact Hall-MHD wave (paper Sec. 4.1), second-order
convergence under diffusive scaling (Sec. 4.3), exact invariants, symmetry, the initial state,
forcing closed forms, and the weak-compressibility level of the validation runs (Sec. 4.2).
"""

import math

import numpy as np
import pytest
import torch

import synthetic
from oracle import analytic, diagnostics, scheme
from oracle.lattice import C, C2, CS2

# Bars on the relative L2 error of u and of b - b0 against the exact wave at 32 nodes per
# wavelength after 200 steps (b0 = 0.1, amplitude 1e-3, nu = eta = 0.01, d_i = 2), per J route and
# branch: the measured error times 1.25 (moment route on beta-: 1.16, the bar it had before).
# Measured (u, b): moment beta+ 2.92% / 4.01%, beta- 8.86% / 10.76%; stencil beta+ 0.39% / 0.61%,
# beta- 0.57% / 0.58%. The moment route's error is a phase lag (test_wave_error_is_a_phase_error):
# its frequency is off by 1.06% (beta+) and 2.15% (beta-), the scheme's second-order dispersion
# error at this resolution (Sec. 4.3: it falls as N^-2), which builds up to 0.03 and 0.09 rad of
# phase over the 200 steps (omega t = 3.2 and 4.8 rad).
TOL_WAVE = {("moment", +1): 0.050, ("moment", -1): 0.125, ("stencil", +1): 0.0076, ("stencil", -1): 0.0073}
# the same wave with the BGK fluid collision (measured moment 4.06%, stencil 0.66%, times 1.25)
TOL_WAVE_BGK = {"moment": 0.051, "stencil": 0.0083}
# the electron-MHD whistler at 32 nodes per wavelength (measured moment 1.26%, stencil 0.87%, times 1.25)
TOL_WAVE_EMHD = {"moment": 0.016, "stencil": 0.011}


def _wave_run(N, steps, amp, b0, d_i, nu=0.01, branch=+1, jmode="stencil", nx=1, ny=1,
              route="closed", collision="central"):
    p = scheme.Params(nx, ny, N, nu, nu, d_i, (0.0, 0.0, b0), jmode, route, collision=collision)
    be = analytic.beta(d_i, 2 * math.pi / N, branch)
    uf = synthetic.wave_field(amp)
    u, gu = synthetic.evaluate(uf, (nx, ny, N))
    b, gb = synthetic.evaluate(synthetic.scaled(uf, be), (nx, ny, N))
    st = scheme.step(scheme.init_state(p, u, b, gu, gb), p, steps)
    return p, st


def _wave_error(N, steps, amp, b0, d_i, **kw):
    p, st = _wave_run(N, steps, amp, b0, d_i, **kw)
    _, U, B, _, _ = scheme.fields(st, p)
    ue, be = analytic.wave(N, steps, amp, b0, p.nu, d_i, kw.get("branch", +1))
    eu = torch.linalg.norm(U[:, :, 0, 0] - ue) / torch.linalg.norm(ue)
    bf = be.clone()
    bf[2] -= b0
    eb = torch.linalg.norm(B[:, :, 0, 0] - be) / torch.linalg.norm(bf)
    return float(eu), float(eb)


@pytest.mark.parametrize("jmode", ["stencil", "moment"])
@pytest.mark.parametrize("branch", [+1, -1])
def test_exact_hall_wave(jmode, branch):
    # 32 nodes per wavelength, b0 = 0.1, amplitude 1e-3, nu = eta = 0.01, d_i = 2, 200 steps
    eu, eb = _wave_error(32, 200, 1e-3, 0.1, 2.0, branch=branch, jmode=jmode)
    tol = TOL_WAVE[(jmode, branch)]
    assert eu < tol and eb < tol, (eu, eb)


def _mode_amplitude(v, k):
    """Complex amplitude of the circularly polarised mode: mean over z of (v_y + i v_x) e^{-ikz}
    (the exact wave's is a e^{-nu k^2 t} e^{-i w t})."""
    z = torch.arange(v.shape[1], dtype=torch.float64)
    return complex(((v[1] + 1j * v[0]) * torch.exp(-1j * k * z)).mean())


@pytest.mark.parametrize("branch", [+1, -1])
def test_wave_error_is_a_phase_error(branch):
    """The moment route's larger exact-wave error is a phase lag from its frequency error, the
    dispersion error of Sec. 4.3 (second order in the grid spacing), not an amplitude error: the
    numerical mode amplitude against the exact one after 200 steps has a phase offset that makes
    up nearly all of the L2 error, and the phase offset grows linearly in time at a relative
    frequency error of 1.06% (beta+) / 2.15% (beta-) (bars x1.25). The stencil route's frequency
    error is below 0.2% on both branches."""
    N, b0, amp, d_i = 32, 0.1, 1e-3, 2.0
    k = 2 * math.pi / N
    w = analytic.frequency(d_i, k, b0, branch)
    bars = {"moment": 0.0106 if branch > 0 else 0.0215, "stencil": 0.0014 if branch > 0 else 0.0009}
    for jmode in ("moment", "stencil"):
        times, phases = [], []
        p, st = _wave_run(N, 0, amp, b0, d_i, branch=branch, jmode=jmode)
        for t in range(40, 201, 40):
            st = scheme.step(st, p, 40)
            _, U, _, _, _ = scheme.fields(st, p)
            ue, _ = analytic.wave(N, t, amp, b0, p.nu, d_i, branch)
            r = _mode_amplitude(U[:, :, 0, 0], k) / _mode_amplitude(ue, k)
            times.append(t)
            phases.append(math.atan2(r.imag, r.real))
        rel_freq = abs(np.polyfit(times, phases, 1)[0] / w)
        eu = float(torch.linalg.norm(U[:, :, 0, 0] - ue) / torch.linalg.norm(ue))
        assert rel_freq < 1.25 * bars[jmode], (jmode, rel_freq)
        if jmode == "moment":
            assert rel_freq > 0.75 * bars[jmode], rel_freq                  # the reading, not just a bound
            assert abs(abs(r) - 1.0) < 0.25 * eu and abs(phases[-1]) > 0.95 * eu, (abs(r), phases[-1], eu)


@pytest.mark.parametrize("jmode", ["stencil", "moment"])
def test_second_order_convergence_diffusive_scaling(jmode):
    # diffusive scaling from (N=32, b0=0.1, a=1e-3, d_i=2, 200 steps): k b0, k a, k d_i and
    # nu k^2 t fixed; the fitted slope of the error against N must be close to -2
    Ns = [16, 32, 64]
    errs = []
    for N in Ns:
        s = N / 32
        eu, eb = _wave_error(N, int(round(200 * s * s)), 1e-3 / s, 0.1 / s, 2.0 * s, jmode=jmode)
        errs.append(max(eu, eb))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert slope < -1.8, (errs, slope)


@pytest.mark.parametrize("jmode", ["stencil", "moment"])
def test_exact_hall_wave_bgk_fluid(jmode):
    # the BGK fluid variant (S = omega I) carries the same Navier-Stokes viscosity: the same
    # exact wave and bound as the central-moment collision
    eu, eb = _wave_error(32, 200, 1e-3, 0.1, 2.0, jmode=jmode, collision="bgk")
    assert eu < TOL_WAVE_BGK[jmode] and eb < TOL_WAVE_BGK[jmode], (eu, eb)


def _emhd_error(N, steps, amp, b0, d_i, jmode, eta=0.01):
    """Electron-MHD run of the exact whistler (fluid at rest at t = 0; the magnetic scheme does
    not see the fluid): relative error of B - b0 after the given steps."""
    p = scheme.Params(1, 1, N, eta, eta, d_i, (0.0, 0.0, b0), jmode, "closed", magnetic="emhd")
    b, gb = synthetic.evaluate(synthetic.wave_field(amp), (1, 1, N))
    z = torch.zeros_like(b)
    st = scheme.step(scheme.init_state(p, z, b, torch.zeros_like(gb), gb), p, steps)
    _, _, B, _, _ = scheme.fields(st, p)
    be = analytic.emhd_wave(N, steps, amp, b0, eta, d_i)
    bf = be.clone()
    bf[2] -= b0
    return float(torch.linalg.norm(B[:, :, 0, 0] - be) / torch.linalg.norm(bf))


@pytest.mark.parametrize("jmode", ["stencil", "moment"])
def test_exact_emhd_whistler_second_order(jmode):
    # electron MHD (Sec. 6): the whistler w = alpha_H b0 k^2 of oracle.analytic, within the wave
    # bound at 32 nodes per wavelength and second order under diffusive scaling
    Ns = [16, 32, 64]
    errs = []
    for N in Ns:
        s = N / 32
        errs.append(_emhd_error(N, int(round(200 * s * s)), 1e-3 / s, 0.1 / s, 2.0 * s, jmode))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert errs[1] < TOL_WAVE_EMHD[jmode] and slope < -1.8, (errs, slope)


def test_translation_invariance():
    # a z-wave on an (nx, ny) = (3, 2) cross-section evolves as on (1, 1), to rounding
    p1, s1 = _wave_run(16, 30, 1e-3, 0.1, 2.0, jmode="stencil")
    p2, s2 = _wave_run(16, 30, 1e-3, 0.1, 2.0, jmode="stencil", nx=3, ny=2)
    assert (s2.f - s1.f).abs().max() < 1e-15
    assert (s2.g - s1.g).abs().max() < 1e-15


def _turbulent_state(n=8, jmode="moment", d_i=2.0, forced=False, seed=0):
    shape = (n, n, n)
    u, gu = synthetic.evaluate(synthetic.shell_field(seed, 1, 2, 0.02), shape)
    b, gb = synthetic.evaluate(synthetic.shell_field(seed + 1, 1, 2, 0.02), shape)
    fu = fb = None
    if forced:
        fu, _ = synthetic.evaluate(synthetic.shell_field(seed + 2, 0, 2, 1e-4, "radius"), shape, gradient=False)
        fb, _ = synthetic.evaluate(synthetic.shell_field(seed + 3, 0, 2, 1e-4, "radius"), shape, gradient=False)
        fu = fu + torch.tensor([2e-5, -1e-5, 3e-5], dtype=torch.float64).view(3, 1, 1, 1)
        fb = fb + torch.tensor([-1e-5, 2e-5, 1e-5], dtype=torch.float64).view(3, 1, 1, 1)
    p = scheme.Params(n, n, n, 0.02, 0.03, d_i, (0.01, -0.02, 0.05), jmode, "closed", fu, fb)
    return p, scheme.init_state(p, u, b, gu, gb)


@pytest.mark.parametrize("jmode", ["moment", "stencil"])
def test_invariants_unforced(jmode):
    p, st = _turbulent_state(jmode=jmode)
    r0 = diagnostics.reductions(st, p)
    st = scheme.step(st, p, 10)
    r1 = diagnostics.reductions(st, p)
    assert abs(r1[9] - r0[9]) < 1e-13 * r0[9]                    # mass
    assert (r1[10:13] - r0[10:13]).abs().max() < 1e-13 * r0[9]    # momentum
    assert (r1[13:16] - r0[13:16]).abs().max() < 1e-13 * r0[9]    # total field


def test_invariants_forced():
    p, st = _turbulent_state(forced=True)
    r0 = diagnostics.reductions(st, p)
    steps = 7
    st = scheme.step(st, p, steps)
    r1 = diagnostics.reductions(st, p)
    assert abs(r1[9] - r0[9]) < 1e-13 * r0[9]
    assert torch.allclose(r1[10:13] - r0[10:13], steps * p.force_u.sum((1, 2, 3)), atol=1e-13, rtol=1e-12)
    assert torch.allclose(r1[13:16] - r0[13:16], steps * p.force_b.sum((1, 2, 3)), atol=1e-13, rtol=1e-12)


def test_uniform_force_accelerates_linearly():
    # a uniform force on a uniform fluid: U(t) = F t / rho exactly
    shape = (2, 2, 2)
    F = torch.tensor([1e-5, -2e-5, 3e-6], dtype=torch.float64).view(3, 1, 1, 1).expand(3, *shape).clone()
    p = scheme.Params(2, 2, 2, 0.05, 0.05, 0.0, (0.0, 0.0, 0.0), "moment", "closed", F, None)
    z = torch.zeros((3,) + shape, dtype=torch.float64)
    st = scheme.init_state(p, z, z)
    st = scheme.step(st, p, 13)
    _, U, _, _, _ = scheme.fields(st, p)
    assert torch.allclose(U, 13 * F, rtol=1e-12, atol=0)


def _kolmogorov_error(N, magnetic=False):
    # steady response to a static sinusoidal source: u = F0 sin(k y) / (nu k^2) x_hat, or with a
    # magnetic source and no flow coupling (d_i = 0, tiny amplitude) B = S0 sin(k y) / (eta k^2)
    k = 2 * math.pi / N
    y = torch.arange(N, dtype=torch.float64).view(1, 1, N, 1)
    src = torch.zeros(3, 1, N, 1, dtype=torch.float64)
    nu = 0.1
    amp = 1e-7
    src[0] = amp * torch.sin(k * y[0])
    fu, fb = (None, src) if magnetic else (src, None)
    p = scheme.Params(1, N, 1, nu, nu, 0.0, (0.0, 0.0, 0.0), "moment", "closed", fu, fb)
    z = torch.zeros((3, 1, N, 1), dtype=torch.float64)
    st = scheme.init_state(p, z, z)
    st = scheme.step(st, p, int(12 / (nu * k * k)))
    _, U, B, _, _ = scheme.fields(st, p)
    got = (B if magnetic else U)[0, 0, :, 0]
    want = amp * torch.sin(k * y[0, 0, :, 0]) / (nu * k * k)
    return float(torch.linalg.norm(got - want) / torch.linalg.norm(want))


@pytest.mark.parametrize("magnetic", [False, True])
def test_forced_steady_state(magnetic):
    e16, e32 = _kolmogorov_error(16, magnetic), _kolmogorov_error(32, magnetic)
    assert e32 < 0.01
    assert e16 / e32 > 3.0          # second order in k


def test_initial_state_moments():
    n = 8
    shape = (n, n, n)
    uf, bf = synthetic.shell_field(4, 1, 2, 0.02), synthetic.shell_field(5, 1, 2, 0.03)
    u, gu = synthetic.evaluate(uf, shape)
    b, gb = synthetic.evaluate(bf, shape)
    p = scheme.Params(n, n, n, 0.01, 0.02, 3.0, (0.0, 0.1, 0.0), "moment", "T")
    st = scheme.init_state(p, u, b, gu, gb)
    rho, U, B, Lam = scheme.moments(st, p)
    B0 = torch.tensor(p.b0, dtype=torch.float64).view(3, 1, 1, 1)
    assert (rho - 1).abs().max() < 1e-15
    assert (U - u).abs().max() < 1e-16
    assert (B - b - B0).abs().max() < 1e-16
    J = scheme.curl_from_gradient(gb)
    V = U - p.d_i * J
    lam0 = torch.einsum("a...,b...->ab...", V, B) - torch.einsum("a...,b...->ab...", B, V)
    assert (Lam - lam0 + (C2 / p.omega_b) * gb).abs().max() < 1e-16
    # the moment route then recovers J = curl B exactly at t = 0
    _, _, _, Jm, _ = scheme.fields(st, p)
    assert (Jm - J).abs().max() < 1e-13
    # deviatoric non-equilibrium second central moment of the fluid
    from oracle.equilibrium import f_mhd_eq
    fneq = st.f - f_mhd_eq(rho, U, B)
    cb = C.view(27, 3, 1, 1, 1) - U.unsqueeze(0)
    K = torch.einsum("iabcd,iebcd,ibcd->aebcd", cb, cb, fneq)
    s = gu + gu.transpose(0, 1)
    div = gu[0, 0] + gu[1, 1] + gu[2, 2]
    P = -(CS2 / p.omega) * (s - (2.0 / 3.0) * div * torch.eye(3, dtype=torch.float64).view(3, 3, 1, 1, 1))
    assert (K - P).abs().max() < 1e-15


def test_xia_density_fluctuation_level():
    # Sec. 4.2: relative density fluctuations of order 1e-7..1e-6 at Ma 0.003..0.01;
    # here N = 16, Ma = 0.007, eps_H = 1 (d_i = N cells), nu = 1e-3 in units of U0 N,
    # b = alpha_+ u + U0 z_hat
    N = 16
    ma = 0.007
    u0 = ma / math.sqrt(3)
    d_i = float(N)
    nu = 1e-3 * u0 * N
    k = 2 * math.pi * 2 / N
    ap = analytic.beta(d_i, k, +1)        # lattice-unit alpha_+ makes each mode an exact wave
    uf = synthetic.xia_field(u0)
    u, gu = synthetic.evaluate(uf, (N, N, N))
    b, gb = synthetic.evaluate(synthetic.scaled(uf, ap), (N, N, N))
    p = scheme.Params(N, N, N, nu, nu, d_i, (0.0, 0.0, u0), "moment", "closed")
    st = scheme.init_state(p, u, b, gu, gb)
    drho = []
    for _ in range(6):
        st = scheme.step(st, p, 25)
        drho.append(float(diagnostics.reductions(st, p)[7]))
    level = float(np.mean(drho))
    assert 1e-8 < level < 1e-5, drho


def test_spectrum_parseval_and_single_mode():
    n = 12
    f = synthetic.shell_field(9, 1, 3, 0.05)
    v, _ = synthetic.evaluate(f, (n, n, n), gradient=False)
    e = diagnostics.spectrum(v, diagnostics.max_shell((n, n, n)))
    assert abs(e.sum() - 0.5 * float((v * v).sum(0).mean())) < 1e-16
    w = synthetic.wave_field(0.3, kz=2)
    v, _ = synthetic.evaluate(w, (n, n, n), gradient=False)
    e = diagnostics.spectrum(v, 6)
    assert abs(e[2] - 0.5 * 0.3 ** 2) < 1e-15 and abs(e.sum() - e[2]) < 1e-15


def test_dissipation_spectrum_sums_to_the_exact_gradient_norm():
    """Parseval for the k^2-weighted spectrum: sum_s D(s) = <|grad v|^2>, with grad v taken from
    the mode sums directly (not through an FFT), on a non-cubic grid; for a solenoidal field on
    a cubic grid it is <|curl v|^2>; a single mode puts q^2 <|v|^2> into its own shell."""
    shape = (10, 12, 14)
    f = synthetic.shell_field(9, 1, 3, 0.05)
    v, g = synthetic.evaluate(f, shape)
    d = diagnostics.dissipation_spectrum(v, diagnostics.max_shell(shape[::-1]))
    ref = float((g * g).sum((0, 1)).mean())
    assert abs(d.sum() - ref) < 1e-14 * ref
    n = 12
    v, g = synthetic.evaluate(f, (n, n, n))
    curl = torch.stack([g[1, 2] - g[2, 1], g[2, 0] - g[0, 2], g[0, 1] - g[1, 0]])
    d = diagnostics.dissipation_spectrum(v, diagnostics.max_shell((n, n, n)))
    ref = float((curl * curl).sum(0).mean())
    assert abs(d.sum() - ref) < 1e-14 * ref
    v, _ = synthetic.evaluate(synthetic.wave_field(0.3, kz=2), (n, n, n), gradient=False)
    d = diagnostics.dissipation_spectrum(v, 6)
    q = 2 * math.pi * 2 / n
    assert abs(d[2] - q * q * 0.3 ** 2) < 1e-15 and abs(d.sum() - d[2]) < 1e-16


def _dft_brute(v):
    """(1/N) sum_x v(x) exp(-2 pi i k . x / n) of a (nz, ny, nx) array by explicit phase matrices."""
    nz, ny, nx = v.shape
    mats = [np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) for n in (nz, ny, nx)]
    return np.einsum("az,by,cx,zyx->abc", mats[0], mats[1], mats[2], v) / v.size


def _transfer_brute(U, gU, B, gB, J, gJ, nshells, d_i):
    """Energy transfer (with the Hall term) from exact node derivatives (mode sums, product rule)
    and explicit DFTs, binned by round(|k|) with the signed index written out in a loop."""
    U, gU, B, gB, J, gJ = [x.numpy() for x in (U, gU, B, gB, J, gJ)]
    adv = np.stack([sum(U[a] * gU[a, b] for a in range(3)) for b in range(3)])
    lor = np.stack([J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0]])
    # d_a (U x B) = d_a U x B + U x d_a B, then curl
    dW = np.stack([np.cross(gU[a], B, axis=0) + np.cross(U, gB[a], axis=0) for a in range(3)])
    curlW = np.stack([dW[1, 2] - dW[2, 1], dW[2, 0] - dW[0, 2], dW[0, 1] - dW[1, 0]])
    dL = np.stack([np.cross(gJ[a], B, axis=0) + np.cross(J, gB[a], axis=0) for a in range(3)])
    curlL = np.stack([dL[1, 2] - dL[2, 1], dL[2, 0] - dL[0, 2], dL[0, 1] - dL[1, 0]])
    F = lambda v: _dft_brute(v)  # noqa: E731
    ta = sum(np.real(np.conj(F(U[b])) * F(adv[b])) for b in range(3))
    tl = -sum(np.real(np.conj(F(U[b])) * F(lor[b])) for b in range(3))
    ti = -sum(np.real(np.conj(F(B[b])) * F(curlW[b])) for b in range(3))
    th = d_i * sum(np.real(np.conj(F(B[b])) * F(curlL[b])) for b in range(3))
    nz, ny, nx = U.shape[1:]
    out = np.zeros((4, nshells))
    signed = lambda k, n: k if k <= (n - 1) // 2 else k - n  # noqa: E731
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                m = (signed(kx, nx), signed(ky, ny), signed(kz, nz))
                s = int(math.floor(math.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2) + 0.5))
                if s < nshells:
                    out[:, s] += (ta[kz, ky, kx], tl[kz, ky, kx], ti[kz, ky, kx], th[kz, ky, kx])
    return out


def test_energy_transfer_matches_brute_force():
    """Fields band-limited to |k_a| <= 1 on a (5, 6, 7) grid: their products stay below every
    axis' Nyquist index, so exact node derivatives (mode sums) and the spectral ones agree and the
    explicit DFT sums must reproduce the oracle to rounding, term by term and shell by shell."""
    shape = (5, 6, 7)
    U, gU = synthetic.evaluate(synthetic.shell_field(41, 1, 1, 0.3), shape)
    B, gB = synthetic.evaluate(synthetic.shell_field(42, 1, 1, 0.2), shape)
    J, gJ = synthetic.evaluate(synthetic.shell_field(43, 1, 1, 0.1), shape)
    ns = diagnostics.max_shell(shape[::-1])
    got = np.stack(diagnostics.energy_transfer(U, B, J, ns, d_i=1.7))
    ref = _transfer_brute(U, gU, B, gB, J, gJ, ns, 1.7)
    scale = np.abs(ref).max()
    assert scale > 1e-4
    assert np.abs(got - ref).max() < 1e-13 * scale


def test_energy_transfer_conserves_energy():
    """Over all shells the nonlinear terms conserve energy: <U . (J x B)> + <B . curl(U x B)> = 0
    when J = curl B, and <U . (U . grad) U> = 0 for a solenoidal U, exact here because the
    products are not aliased (|k_a| <= 4 on 9 nodes, |k_a| <= 2 on (5, 6, 7))."""
    shape = (5, 6, 7)
    U, _ = synthetic.evaluate(synthetic.shell_field(44, 1, 1, 0.3), shape)
    B, gB = synthetic.evaluate(synthetic.shell_field(45, 1, 1, 0.2), shape)
    J = torch.stack([gB[1, 2] - gB[2, 1], gB[2, 0] - gB[0, 2], gB[0, 1] - gB[1, 0]])
    ta, tl, ti = diagnostics.energy_transfer(U, B, J, diagnostics.max_shell(shape[::-1]))
    assert np.abs(tl).sum() > 1e-5 and abs(tl.sum() + ti.sum()) < 1e-14 * np.abs(tl).sum()
    # the Hall term conserves the energy on its own: alpha_H <J . (J x B)> = 0 for J = curl B;
    # B in shells 1 and 2 (a field in one shell only has nothing to move between shells), on a
    # grid where the products of |k_a| <= 2 modes are not aliased
    shape = (9, 10, 11)
    B, gB = synthetic.evaluate(synthetic.shell_field(47, 1, 2, 0.2), shape)
    J = torch.stack([gB[1, 2] - gB[2, 1], gB[2, 0] - gB[0, 2], gB[0, 1] - gB[1, 0]])
    *_, th = diagnostics.energy_transfer(B, B, J, diagnostics.max_shell(shape[::-1]), d_i=2.5)
    assert np.abs(th).sum() > 1e-6 and abs(th.sum()) < 1e-14 * np.abs(th).sum()
    n = 9
    U, _ = synthetic.evaluate(synthetic.shell_field(46, 1, 2, 0.3), (n, n, n))
    ta, _, _ = diagnostics.energy_transfer(U, U, U, diagnostics.max_shell((n, n, n)))
    assert np.abs(ta).sum() > 1e-4 and abs(ta.sum()) < 1e-14 * np.abs(ta).sum()
