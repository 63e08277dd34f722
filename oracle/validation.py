"""Error measures of the paper's wave validation (Sec. 4.3) -- TEST INFRASTRUCTURE ONLY.

All three compare a numerical time series u(t) of one velocity component at a fixed node with
the exact solution u_bar(t) at the same node:

* dispersion error (eq. dispersion_error): with t_i and t_bar_i the times of the successive
  local maxima of u and u_bar, eps_phi = 1 - (1/M) sum_i (t_{i+1} - t_i) / (t_bar_{i+1} - t_bar_i)
  over M periods;
* dissipation error (eq. dissipation_error_new): after synchronising the phases, the rms over
  M periods of the relative difference of the magnitudes. Reading: the magnitudes compared are
  the values at the local maxima, u(t_i) against u_bar(t_bar_i), i.e. each period's maximum of
  the numerical solution against the exact one;
* viscosity error (eq. viscosity_error): the effective viscosity nu_eff of the numerical
  damping exp(-nu_eff k^2 t), taken from a least-squares fit of log u(t_i) against t_i, and
  eps_nu = (nu_eff - nu) / nu.

Maxima are located between samples by the parabola through the largest sample and its two
neighbours (exact for a sampled quadratic, second order in the sampling interval otherwise).
"""

from __future__ import annotations

import math

import numpy as np


def local_maxima(t, u):
    """(times, values) of the interior local maxima of a sampled series, refined by parabolas."""
    t = np.asarray(t, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    times, values = [], []
    for j in range(1, len(u) - 1):
        if u[j] > u[j - 1] and u[j] >= u[j + 1]:
            h = t[j + 1] - t[j]
            if abs((t[j] - t[j - 1]) - h) > 1e-9 * abs(h):
                raise ValueError("local_maxima needs uniform sampling")
            den = u[j - 1] - 2.0 * u[j] + u[j + 1]
            s = 0.5 * (u[j - 1] - u[j + 1]) / den if den != 0 else 0.0
            times.append(t[j] + s * h)
            values.append(u[j] - 0.25 * (u[j - 1] - u[j + 1]) * s)
    return np.array(times), np.array(values)


def dispersion_error(t, u, u_bar, periods):
    """eps_phi over the first `periods` periods (needs periods + 1 maxima in both series)."""
    tn, _ = local_maxima(t, u)
    te, _ = local_maxima(t, u_bar)
    m = periods
    if len(tn) < m + 1 or len(te) < m + 1:
        raise ValueError(f"need {m + 1} maxima, found {len(tn)} and {len(te)}")
    ratios = [(tn[i + 1] - tn[i]) / (te[i + 1] - te[i]) for i in range(m)]
    return 1.0 - sum(ratios) / m


def dissipation_error(t, u, u_bar, periods):
    """eps_r over the first `periods` maxima of each series, compared period by period."""
    _, vn = local_maxima(t, u)
    _, ve = local_maxima(t, u_bar)
    m = periods
    if len(vn) < m or len(ve) < m:
        raise ValueError(f"need {m} maxima, found {len(vn)} and {len(ve)}")
    return math.sqrt(sum(((vn[i] - ve[i]) / ve[i]) ** 2 for i in range(m)) / m)


def viscosity_error(t, u, k, nu, periods):
    """eps_nu from the damping of the first `periods` + 1 maxima of u (wavenumber k)."""
    tn, vn = local_maxima(t, u)
    m = periods + 1
    if len(vn) < m:
        raise ValueError(f"need {m} maxima, found {len(vn)}")
    slope = np.polyfit(tn[:m], np.log(vn[:m]), 1)[0]
    nu_eff = -slope / (k * k)
    return (nu_eff - nu) / nu
