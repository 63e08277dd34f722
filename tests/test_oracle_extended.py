"""Pins of the extended-precision evaluation (oracle/extended.py) against the FP64 oracle,
and the FP64 oracle's rounding floor that it exposes."""

import numpy as np
import pytest

from oracle import extended, scheme

from parity_helpers import Case, extended_run, inputs, oracle_params, oracle_run


def _rel(st, p, ref):
    rest = scheme.rest_state(p)
    xf, xg = ref
    of = (st.f - rest.f).numpy().astype(np.longdouble)
    og = (st.g - rest.g).numpy().astype(np.longdouble)
    num = ((of - xf) ** 2).sum() + ((og - xg) ** 2).sum()
    return float(np.sqrt(num / ((xf ** 2).sum() + (xg ** 2).sum())))


@pytest.mark.parametrize("case", [Case(8, 7, 6, jmode="moment", seed=11), Case(8, 7, 6, jmode="stencil", seed=11),
                                  Case(6, 6, 6, jmode="stencil", forced=True, seed=5, d_i=4.0),
                                  Case(7, 6, 5, jmode="moment", forced=True, seed=6, collision="bgk"),
                                  Case(7, 6, 5, jmode="moment", forced=True, seed=8, magnetic="emhd"),
                                  Case(7, 6, 5, jmode="stencil", seed=10, collision="bgk", magnetic="emhd")])
def test_extended_agrees_with_fp64_oracle(case):
    for steps, tol in ((0, 1e-14), (3, 1e-13)):
        p, st = oracle_run(case, steps, route="T")
        assert _rel(st, p, extended_run(case, steps)) < tol


def test_fp64_oracle_floor_is_reported():
    # after 100 steps the FP64 oracle sits a few 1e-12 from the extended evaluation of the
    # same definition: its own rounding, amplified by the flow. GPU FP64 parity is therefore
    # measured against the extended evaluation.
    case = Case(8, 7, 6, jmode="moment", seed=11)
    p, st = oracle_run(case, 100)
    floor = _rel(st, p, extended_run(case, 100))
    print("FP64 oracle floor after 100 steps:", floor)
    assert 1e-14 < floor < 2e-11


def test_extended_rest_state_and_invariants():
    case = Case(6, 5, 4, jmode="moment", seed=2)
    u, gu, b, gb, _, _ = inputs(case)
    xp = extended.Params(oracle_params(case))
    f, g = extended.init_state(xp, u, b, gu, gb)
    m0 = f.sum()
    B0 = g.sum(axis=(0, 2, 3, 4))
    f, g = extended.step(f, g, xp, 5)
    assert abs(f.sum() - m0) < 1e-16 * m0
    assert np.abs(g.sum(axis=(0, 2, 3, 4)) - B0).max() < 1e-17 * m0
    fr, gr = extended.rest_state(xp, (4, 5, 6))
    rest = scheme.rest_state(oracle_params(case))
    assert np.abs(fr - rest.f.numpy()).max() < 1e-17
