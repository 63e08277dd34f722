"""The Orszag-Tang vortex, the initial condition of the paper's turbulence runs (Sec. 4.4, Sec. 5):
time series of the energies and of the dissipation rate, and the energy budget they must close.

Lattice units: u amplitude U0 = Ma / sqrt(3) with Ma = 0.025 (the Mach number of the paper's
comparison with a pseudo-spectral code), B amplitude 0.8 U0, b0 = 0, rho = 1, reference time
tau0 = (n / 2 pi) / U0 (the box is 2 pi reference lengths), nu = eta from the initial Reynolds
number Re0 = 2 U0 n / nu (initial rms velocity 2 U0, box length n).

Energy budget. In incompressible MHD the energy E = 1/2 <|u|^2 + |B|^2> changes only by
dissipation, dE/dt = -eps with eps = nu <|grad u|^2> + eta <|grad B|^2>, which is nu sum D_u +
eta sum D_B over the dissipation spectra; the Hall term conserves E (J . (J x B) = 0). The
lattice scheme adds two effects, both removing energy from E: the start (rho = 1) is not in
pressure balance, so sound takes up and exchanges back an energy of the order of the squared rms
Mach number times E, (2 Ma)^2 E(0); and the scheme's own dissipation exceeds nu k^2 at second
order in k dx (3% at 24^3 in the oracle, falling as n^-2). The missing energy
E(0) - E(t) - int_0^t eps dt is therefore positive and below 4 Ma^2 E(0) + 0.02 int_0^t eps dt at
every sample (measured: the sound share peaks near 2.5 Ma^2 E(0) early on; at the end of the
runs the missing energy is 0.8-1.0% of int eps at 64^3 and 512^3).

FP32 storage against FP64: a 2^-24 rounding of the stored deviations per step random-walks to
6e-8 sqrt(S) of the velocity after S steps, 2 x that in E; over S = 1412 steps (2 tau0 at 64^3)
that is 4.5e-6, and the bar takes a factor 10 (the flow at Re0 = 200 is laminar-to-transitional
over this time, so it does not amplify the difference much).

The 512^3 FP64 run to beyond the dissipation peak is opt-in (FLAME_LARGE=1): Re0 = 3200 reaches
Re = 1122 at the peak (the paper's comparison run: about 1600) at t = 2.6 tau0. The same run at
128^3 (Re0 = 800) runs by default, as does the Hall-parameter study at 128^3."""

import math
import os

import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

MA = 0.025


def ot_run(n, storage, re0, eps_h, tau_end, samples, log=None, spectra=None):
    """Run the Orszag-Tang vortex on n^3 to tau_end reference times; (params, rows) with rows of
    (step, t / tau0, E, eps, E_kin, E_mag, <|J|^2>, non-finite nodes, Re). Re = u_rms L / nu with
    u_rms = <|u|^2>^(1/2) and the integral scale L = n sum_s E_u(s) / s / sum_s E_u(s) in cells
    (Sec. 4.4, with the box of n cells as 2 pi reference lengths)."""
    from paper_2212_11024_amd.solver import Solver
    u0 = MA / math.sqrt(3.0)
    nu = 2.0 * u0 * n / re0
    tau0 = (n / (2.0 * math.pi)) / u0
    fu, fb = synthetic.orszag_tang(u0, 0.8 * u0)
    u, gu = synthetic.evaluate(fu, (n, n, n), "cuda")
    b, gb = synthetic.evaluate(fb, (n, n, n), "cuda")
    s = Solver(n, n, n, nu, nu, eps_h * n, (0.0, 0.0, 0.0), storage, "moment", "aa", u, b, gu, gb)
    del u, gu, b, gb
    torch.cuda.empty_cache()
    ns = n // 2 + 1
    every = max(1, int(round(tau_end * tau0 / samples)))
    rows = []
    for i in range(samples + 1):
        red = s.reduce(allow_nonfinite=True)
        eps = nu * float(s.dissipation_spectrum("u", ns).sum() + s.dissipation_spectrum("B", ns).sum())
        eu = s.spectrum("u", ns)[1:]
        scale = n * float((eu / torch.arange(1, ns, dtype=eu.dtype)).sum() / eu.sum())
        re = math.sqrt(2.0 * float(red[0])) * scale / nu
        rows.append((i * every, i * every / tau0, float(red[0] + red[1]), eps, float(red[0]), float(red[1]),
                     float(red[3]), int(red[8]), re))
        if spectra is not None:
            spectra.append((eu.numpy().copy(), s.spectrum("B", ns)[1:].numpy().copy()))
        if log:
            log(rows[-1])
        if i < samples:
            s.step(every)
    s.close()
    return {"nu": nu, "tau0": tau0, "every": every}, rows


def test_turbulence_summary_matches_its_parts():
    """Solver.turbulence against the same quantities assembled from the reductions and spectra."""
    from paper_2212_11024_amd.solver import Solver
    n = 32
    u0 = MA / math.sqrt(3.0)
    fu, fb = synthetic.orszag_tang(u0, 0.8 * u0)
    u, gu = synthetic.evaluate(fu, (n, n, n), "cuda")
    b, gb = synthetic.evaluate(fb, (n, n, n), "cuda")
    s = Solver(n, n, n, 0.01, 0.02, 0.5, (0.0, 0.0, 0.0), "f64", "moment", "aa", u, b, gu, gb)
    s.step(50)
    t = s.turbulence()
    ns = n // 2 + 1
    red = s.reduce()
    eps = 0.01 * float(s.dissipation_spectrum("u", ns).sum()) + 0.02 * float(s.dissipation_spectrum("B", ns).sum())
    eu = s.spectrum("u", ns)[1:]
    scale = n * float((eu / torch.arange(1, ns, dtype=torch.float64)).sum() / eu.sum())
    assert t["E_kin"] == float(red[0]) and t["E_mag"] == float(red[1])
    assert abs(t["eps"] / eps - 1) < 1e-12 and abs(t["integral_scale"] / scale - 1) < 1e-12
    assert abs(t["Re"] - math.sqrt(2 * float(red[0])) * scale / 0.01) < 1e-9 * t["Re"]
    # against the oracle's summary of the same run (its fields after the same 50 steps)
    from oracle import diagnostics, scheme
    p = scheme.Params(n, n, n, 0.01, 0.02, 0.5, (0.0, 0.0, 0.0), "moment", "closed")
    st = scheme.step(scheme.init_state(p, u.cpu(), b.cpu(), gu.cpu(), gb.cpu()), p, 50)
    _, ou, oB, _, _ = scheme.fields(st, p)
    ref = diagnostics.turbulence_summary(ou, oB, 0.01, 0.02)
    for key in ("E_kin", "E_mag", "eps", "u_rms", "integral_scale", "Re"):
        assert abs(t[key] - ref[key]) <= 1e-10 * abs(ref[key]), (key, t[key], ref[key])
    # the Orszag-Tang velocity lives in shell 1 at t = 0: L is the box
    s0 = Solver(n, n, n, 0.01, 0.02, 0.5, (0.0, 0.0, 0.0), "f64", "moment", "aa", u, b, gu, gb)
    assert abs(s0.turbulence()["integral_scale"] - n) < 1e-9 * n
    s.close()
    s0.close()


def budget(rows):
    """(t / tau0, missing energy E(0) - E(t) - int_0^t eps dt, int_0^t eps dt) at every sample
    after the first, with the trapezoid rule between samples."""
    out, integral = [], 0.0
    for a, b in zip(rows, rows[1:]):
        integral += 0.5 * (a[3] + b[3]) * (b[0] - a[0])
        out.append((b[1], rows[0][2] - b[2] - integral, integral))
    return out


def check_budget(rows, tag):
    e0 = rows[0][2]
    ratios = []
    for t, missing, integral in budget(rows):
        assert 0.0 < missing < 4.0 * MA * MA * e0 + 0.02 * integral, (t, missing, integral)
        ratios.append(missing / integral)
    print(f"[{tag}] missing energy / int eps: {ratios[len(ratios) // 4]:.4f} at a quarter of the run, "
          f"{ratios[-1]:.4f} at the end", flush=True)


@pytest.mark.parametrize("eps_h", [0.0, 0.01])
def test_energy_budget_closes_64(eps_h):
    print(f"[orszag-tang] 64^3 FP64 and FP32, Re0 = 200, eps_h = {eps_h}, 2 tau0", flush=True)
    runs = {st: ot_run(64, st, 200.0, eps_h, 2.0, 40) for st in ("f64", "f32")}
    for st, (prm, rows) in runs.items():
        assert all(r[7] == 0 for r in rows)
        assert rows[-1][2] < 0.6 * rows[0][2]          # the vortex decays
        check_budget(rows, f"orszag-tang {st}")
    e64 = torch.tensor([r[2] for r in runs["f64"][1]])
    e32 = torch.tensor([r[2] for r in runs["f32"][1]])
    rel = float(((e32 - e64).abs() / e64).max())
    print(f"[orszag-tang]   FP32 vs FP64 energy: max relative {rel:.2e}", flush=True)
    assert rel < 4.5e-5


def test_orszag_tang_128_to_dissipation_peak():
    """The paper's Orszag-Tang run to past its dissipation peak at 128^3 (the 512^3 run below is
    opt-in): FP64, Re0 = 800, d_i = 0, to 3 tau0 (4233 steps). Checked: finite throughout, the
    peak of the dissipation rate inside the run, the energy budget at every sample (bound as in
    the module docstring), and the FP32-storage run tracking it. Measured: the peak at 1.41 tau0
    (Re 395), missing energy 1.3% of int eps at a quarter of the run and 1.9% at the end, FP32
    against FP64 at most 2.0e-5 relative on E and 3.6e-5 on eps over the run; the bars take ten
    times those (the runs are bitwise reproducible, so the factor only covers a change of the
    kernels' rounding order)."""
    n = 128
    print("[orszag-tang 128] FP64 and FP32, Re0 = 800, d_i = 0, to 3 tau0", flush=True)
    prm, rows = ot_run(n, "f64", 800.0, 0.0, 3.0, 60)
    assert all(r[7] == 0 for r in rows)
    ip = max(range(len(rows)), key=lambda i: rows[i][3])
    peak = rows[ip]
    print(f"[orszag-tang 128] nu {prm['nu']:.4e}, tau0 {prm['tau0']:.1f} steps; dissipation peak at "
          f"t/tau0 = {peak[1]:.3f}, eps = {peak[3]:.4e}, Re = {peak[8]:.0f}", flush=True)
    check_budget(rows, "orszag-tang 128")
    assert 0 < peak[1] < 3.0 - 1e-9
    _, rows32 = ot_run(n, "f32", 800.0, 0.0, 3.0, 60)
    assert all(r[7] == 0 for r in rows32)
    de = max(abs(a[2] - b[2]) / b[2] for a, b in zip(rows32, rows))
    dps = max(abs(a[3] - b[3]) / b[3] for a, b in zip(rows32, rows))
    print(f"[orszag-tang 128] FP32 vs FP64 over the run: energy {de:.2e}, dissipation {dps:.2e} (max relative)",
          flush=True)
    assert de < 2e-4 and dps < 4e-4


@pytest.mark.skipif(os.environ.get("FLAME_LARGE") != "1", reason="opt-in 512^3 run (FLAME_LARGE=1)")
def test_orszag_tang_512_to_dissipation_peak():
    n = 512
    print("[orszag-tang] 512^3 FP64, Re0 = 3200, d_i = 0, to 3 tau0", flush=True)

    def log(r):
        print(f"[orszag-tang 512] step {r[0]} t/tau0 {r[1]:.3f} E {r[2]:.6e} eps {r[3]:.6e} E_kin {r[4]:.6e} "
              f"E_mag {r[5]:.6e} <J^2> {r[6]:.6e} bad {r[7]} Re {r[8]:.0f}", flush=True)

    spec = {"f64": [], "f32": []}
    prm, rows = ot_run(n, "f64", 3200.0, 0.0, 3.0, 60, log, spec["f64"])
    assert all(r[7] == 0 for r in rows)
    ip = max(range(len(rows)), key=lambda i: rows[i][3])
    peak = rows[ip]
    print(f"[orszag-tang 512] nu {prm['nu']:.4e} tau0 {prm['tau0']:.1f} steps; dissipation peak at "
          f"t/tau0 = {peak[1]:.3f}, eps = {peak[3]:.4e}, Re = {peak[8]:.0f}", flush=True)
    check_budget(rows, "orszag-tang 512")
    assert 0 < peak[1] < 3.0 - 1e-9                      # the peak lies inside the run
    # shell spectra at the peak, normalised by their totals (the paper's comparison at the peak)
    k = np.arange(1, len(spec["f64"][ip][0]) + 1)
    for name, e in (("E_u", spec["f64"][ip][0]), ("E_B", spec["f64"][ip][1])):
        en = e / e.sum()
        fit = (k >= 4) & (k <= 24)
        slope = np.polyfit(np.log(k[fit]), np.log(en[fit]), 1)[0]
        print(f"[orszag-tang 512] {name}(k) / E at the peak, k = 1..32: "
              + " ".join(f"{x:.3e}" for x in en[:32]) + f"; fitted slope over k = 4..24: {slope:.2f}", flush=True)
    # the same run with FP32 storage: energies and the spectra at the FP64 peak
    prm32, rows32 = ot_run(n, "f32", 3200.0, 0.0, 3.0, 60,
                           lambda r: print(f"[orszag-tang 512 FP32] step {r[0]} E {r[2]:.6e} eps {r[3]:.6e}",
                                           flush=True), spec["f32"])
    assert all(r[7] == 0 for r in rows32)
    de = max(abs(a[2] - b[2]) / b[2] for a, b in zip(rows32, rows))
    dps = max(abs(a[3] - b[3]) / b[3] for a, b in zip(rows32, rows))
    su = np.abs(spec["f32"][ip][0][:8] / spec["f64"][ip][0][:8] - 1).max()
    sb = np.abs(spec["f32"][ip][1][:8] / spec["f64"][ip][1][:8] - 1).max()
    print(f"[orszag-tang 512] FP32 vs FP64 over the run: energy {de:.2e}, dissipation {dps:.2e} (max relative); "
          f"shells 1..8 at the peak: E_u {su:.2e}, E_B {sb:.2e}", flush=True)


def test_scale_by_scale_budget_64():
    """The band budget of Sec. 4.4 (eq. mhd_en_trans): over [0, t], the change of the energy in
    shells s < k equals -int (S_MHD(k) + D(k)) dt, with S from the transfer terms and D from the
    dissipation spectra, for every band k. Bound per band and sample: the sound share of the
    total budget (4 Ma^2 E(0), see above) plus 3% of the largest of the three integrals, which
    covers the scheme's excess dissipation, the pressure work of the weakly compressible flow and
    the moment route's J against the spectral curl of B (measured: at most 1.2% from 0.5 tau0 on
    at 64^3, 1.9% at 128^3)."""
    from paper_2212_11024_amd.solver import Solver
    n = 64
    u0 = MA / math.sqrt(3.0)
    nu = 2.0 * u0 * n / 200.0
    tau0 = (n / (2.0 * math.pi)) / u0
    fu, fb = synthetic.orszag_tang(u0, 0.8 * u0)
    u, gu = synthetic.evaluate(fu, (n, n, n), "cuda")
    b, gb = synthetic.evaluate(fb, (n, n, n), "cuda")
    print("[orszag-tang] 64^3 FP64 band budget, Re0 = 200, d_i = 0, 2 tau0", flush=True)
    s = Solver(n, n, n, nu, nu, 0.0, (0.0, 0.0, 0.0), "f64", "moment", "aa", u, b, gu, gb)
    ns = n // 2 + 1
    samples = 40
    every = int(round(2.0 * tau0 / samples))
    rec = []
    for i in range(samples + 1):
        E = s.spectrum("u", ns) + s.spectrum("B", ns)
        D = nu * (s.dissipation_spectrum("u", ns) + s.dissipation_spectrum("B", ns))
        T = s.energy_transfer(ns).sum(0)
        rec.append((i * every, E, D, T))
        if i < samples:
            s.step(every)
    s.close()
    e0 = float(rec[0][1].sum())
    worst = 0.0
    for k in (2, 3, 4, 6, 8, 12, 16, ns):
        int_s = int_d = 0.0
        for a, b_ in zip(rec, rec[1:]):
            dt = b_[0] - a[0]
            int_s += 0.5 * float(a[3][:k].sum() + b_[3][:k].sum()) * dt
            int_d += 0.5 * float(a[2][:k].sum() + b_[2][:k].sum()) * dt
            d_e = float(b_[1][:k].sum() - rec[0][1][:k].sum())
            big = max(abs(d_e), abs(int_s), abs(int_d))
            miss = abs(d_e + int_s + int_d)
            assert miss < 4.0 * MA * MA * e0 + 0.03 * big, (k, b_[0] / tau0, d_e, int_s, int_d)
            if b_[0] >= 0.5 * tau0:
                worst = max(worst, miss / big)
    print(f"[orszag-tang]   band budget: largest residual from 0.5 tau0 on {worst:.4f} of the largest term",
          flush=True)


def hall_study(n, re0, d_cells, kfit, tau_end=3.5, samples=50):
    """Orszag-Tang runs at n^3 (FP64, Ma = 0.025) for each Hall parameter d_i (cells): per run, the
    time of the dissipation peak (tau0), E_B / E_u over the shells k > kfit[0] at the peak and the
    magnetic spectral slope fitted over kfit."""
    res = []
    for d_i in d_cells:
        spec = []
        print(f"[orszag-tang hall] {n}^3 FP64, Re0 = {re0:.0f}, d_i = {d_i}", flush=True)
        prm, rows = ot_run(n, "f64", re0, d_i / n, tau_end, samples, None, spec)
        assert all(r[7] == 0 for r in rows)
        ip = max(range(len(rows)), key=lambda i: rows[i][3])
        eu, eb = spec[ip]
        k = np.arange(1, len(eu) + 1)
        m = (k >= kfit[0]) & (k <= kfit[1])
        res.append((rows[ip][1], float(eb[k > kfit[0]].sum() / eu[k > kfit[0]].sum()),
                    float(np.polyfit(np.log(k[m]), np.log(eb[m]), 1)[0])))
        print(f"[orszag-tang hall] d_i = {d_i}: peak at {res[-1][0]:.3f} tau0 (Re {rows[ip][8]:.0f}), "
              f"E_B/E_u (k > {kfit[0]}) {res[-1][1]:.2f}, magnetic slope (k = {kfit[0]}..{kfit[1]}) "
              f"{res[-1][2]:.2f}", flush=True)
    return res


def test_hall_parameter_changes_the_turbulence_128():
    """The Hall trends of Sec. 5 (see the 256^3 study below) at 128^3, Re0 = 800, between the MHD
    run and d_i = 4 cells (k_H = n / (2 pi d_i) = 5, as for d_i = 8 at 256^3): at the dissipation
    peak the Hall run's small scales are more magnetic, with a shallower magnetic spectrum.
    Measured: E_B / E_u over shells k > 10 of 2.86 (MHD) and 4.38 (Hall), magnetic slopes over
    k = 10..30 of -6.20 and -4.79. The earlier peak of the Hall run seen at 256^3 does not show
    at this Reynolds number (both peak at 1.40 tau0, within the sampling of 0.07 tau0), so here
    the peak is only required not to come later."""
    peaks, ratio, slope = zip(*hall_study(128, 800.0, (0.0, 4.0), (10, 30)))
    assert peaks[1] <= peaks[0]
    assert ratio[1] > 1.3 * ratio[0]
    assert slope[1] > slope[0] + 1.0


@pytest.mark.skipif(os.environ.get("FLAME_LARGE") != "1", reason="opt-in 256^3 Hall study (FLAME_LARGE=1)")
def test_hall_parameter_changes_the_turbulence_256():
    """The Hall-MHD trends the paper reports for its Orszag-Tang runs (Sec. 5), at 256^3 (FP64,
    Ma = 0.025, Re0 = 1600, about 600-700 at the peak) for d_i = 0, 2, 4, 8 cells: a larger Hall
    parameter makes the turbulence develop faster (earlier dissipation peak), and at the peak the
    sub-ion scales become magnetically dominated with a shallower magnetic spectrum (energy held
    beyond k_H = n / (2 pi d_i) instead of the MHD run's steep dissipation range). Measured: peak
    at 2.46 / 2.46 / 2.39 / 2.17 tau0; E_B / E_u over shells k > 20 of 2.2 / 2.2 / 2.8 / 5.8;
    magnetic slope over k = 20..60 of -6.9 / -6.4 / -5.5 / -4.7."""
    peaks, ratio, slope = zip(*hall_study(256, 1600.0, (0.0, 2.0, 4.0, 8.0), (20, 60)))
    assert peaks[3] < 0.95 * peaks[0]
    assert all(a <= b for a, b in zip(ratio, ratio[1:])) and ratio[3] > 2 * ratio[0]
    assert all(a < b for a, b in zip(slope, slope[1:]))
