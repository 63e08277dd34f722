"""Pins of the wave-validation error measures (oracle/validation.py; paper Sec. 4.3, eqs.
dispersion_error, dissipation_error_new and viscosity_error) on damped cosines, whose maxima
have closed forms: u = A exp(-g t) cos(w t + p) peaks where tan(w t + p) = -g / w, i.e. at
t_m = (2 pi m - atan(g / w) - p) / w, with the values A exp(-g t_m) / sqrt(1 + (g / w)^2)."""

import math

import numpy as np
import pytest

from oracle import validation as V


def _damped(t, a, g, w, p=0.0):
    return a * np.exp(-g * t) * np.cos(w * t + p)


def _peaks(a, g, w, p, m):
    t = np.array([(2 * math.pi * i - math.atan(g / w) - p) / w for i in range(m)])
    return t, a * np.exp(-g * t) / math.sqrt(1 + (g / w) ** 2)


def test_local_maxima_of_a_sampled_parabola_is_exact():
    t = np.arange(0.0, 10.0, 0.5)
    u = -(t - 3.3) ** 2 + 2.0
    tm, vm = V.local_maxima(t, u)
    assert len(tm) == 1 and abs(tm[0] - 3.3) < 1e-12 and abs(vm[0] - 2.0) < 1e-12


def test_maxima_of_a_damped_cosine():
    w, g, p = 2 * math.pi / 97.0, 1.3e-3, 0.4
    t = np.arange(0.0, 1200.0, 0.25)
    tm, vm = V.local_maxima(t, _damped(t, 0.7, g, w, p))
    te, ve = _peaks(0.7, g, w, p, 14)
    te, ve = te[te > 0][: len(tm)], ve[te > 0][: len(tm)]
    assert np.abs(tm - te).max() < 1e-4 and np.abs(vm / ve - 1).max() < 1e-8


def test_dispersion_error_of_a_detuned_wave():
    # numerical frequency w' against exact w: every period ratio is w / w', eps_phi = 1 - w / w'
    w, wn, g = 2 * math.pi / 200.0, 2 * math.pi / 198.0, 5e-4
    t = np.arange(0.0, 2500.0, 0.5)
    eps = V.dispersion_error(t, _damped(t, 1.0, g, wn), _damped(t, 1.0, g, w), 10)
    assert abs(eps - (1 - w / wn)) < 1e-7


def test_dissipation_error_of_an_overdamped_wave():
    # same frequency, damping g' > g: per-period amplitude ratios from the closed-form peaks
    w, g, gn = 2 * math.pi / 150.0, 4e-4, 5e-4
    t = np.arange(0.0, 2000.0, 0.25)
    eps = V.dissipation_error(t, _damped(t, 1.0, gn, w), _damped(t, 1.0, g, w), 10)
    _, vn = _peaks(1.0, gn, w, 0.0, 12)
    _, ve = _peaks(1.0, g, w, 0.0, 12)
    vn, ve = vn[1:11], ve[1:11]            # the first peak at t < 0 is not sampled
    ref = math.sqrt(np.mean(((vn - ve) / ve) ** 2))
    assert abs(eps - ref) < 1e-7 and eps > 0.01


@pytest.mark.parametrize("excess", [0.0, 0.03, -0.02])
def test_viscosity_error_recovers_the_damping(excess):
    k, nu = 2 * math.pi / 32, 0.01
    g = nu * (1 + excess) * k * k
    t = np.arange(0.0, 4000.0, 0.5)
    eps = V.viscosity_error(t, _damped(t, 1e-3, g, 2 * math.pi / 389.0), k, nu, 8)
    assert abs(eps - excess) < 1e-6


def test_turbulence_summary_closed_forms():
    """The turbulence summary of Sec. 4.4 on fields with closed-form answers: a single sine mode
    of shell s gives L = n / s, eps = nu a^2 q^2 / 2 with q = 2 pi s / n, E_kin = a^2 / 4 and
    Re = (a / sqrt 2) L / nu; two modes of energies E1 (shell 1) and E2 (shell 2) give
    L = n (E1 + E2 / 2) / (E1 + E2); B's energy is measured from b0."""
    import math

    import torch

    from oracle import diagnostics as D
    n, nu, eta = 16, 0.01, 0.02
    x = torch.arange(n, dtype=torch.float64)
    for s in (1, 3):
        a = 0.03
        u = torch.zeros(3, n, n, n, dtype=torch.float64)
        u[1] = a * torch.sin(2 * math.pi * s * x / n).view(1, 1, n)
        B = torch.zeros_like(u)
        B[2] += 0.1
        t = D.turbulence_summary(u, B, nu, eta, b0=(0.0, 0.0, 0.1))
        q = 2 * math.pi * s / n
        assert abs(t["integral_scale"] - n / s) < 1e-12 * n
        assert abs(t["eps"] - nu * a * a * q * q / 2) < 1e-12 * nu * a * a * q * q
        assert abs(t["E_kin"] - a * a / 4) < 1e-15 and t["E_mag"] == 0.0
        assert abs(t["Re"] - (a / math.sqrt(2)) * (n / s) / nu) < 1e-9 * t["Re"]
    a1, a2 = 0.02, 0.05
    u = torch.zeros(3, n, n, n, dtype=torch.float64)
    u[0] = (a1 * torch.cos(2 * math.pi * x / n)).view(1, n, 1) + (a2 * torch.sin(4 * math.pi * x / n)).view(n, 1, 1)
    e1, e2 = a1 * a1 / 4, a2 * a2 / 4
    t = D.turbulence_summary(u, torch.zeros_like(u), nu, eta)
    assert abs(t["integral_scale"] - n * (e1 + e2 / 2) / (e1 + e2)) < 1e-12 * n
