"""Seeded input generator (shared by both sides) and the printed lattice listing."""

import os
from fractions import Fraction

import numpy as np

import synthetic
from oracle.lattice import C, C2, W, WM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d3q27_app_a.txt")


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        rows[key] = [float(Fraction(v)) for v in vals]
    return rows


def test_oracle_lattice_matches_printed_listing():
    g = _golden()
    assert C[:, 0].tolist() == g["cx"] and C[:, 1].tolist() == g["cy"] and C[:, 2].tolist() == g["cz"]
    by_speed = {int(s): float(w) for s, w in zip((C * C).sum(1), W)}
    assert [by_speed[s] for s in range(4)] == g["w"]
    assert float(WM[0]) == g["W"][0] and float(WM[1]) == g["W"][1] and C2 == g["C2"][0]


def test_mode_counts_and_rms():
    assert len(synthetic.half_space_wavevectors(1, 4)) == 194
    assert len(synthetic.half_space_wavevectors(0, 2, "radius")) == 16
    f = synthetic.shell_field(0, 1, 4, 0.02)
    assert abs(f.rms - 0.02) < 1e-15
    v, g = synthetic.evaluate(f, (10, 12, 14))
    assert abs(float((v * v).sum(0).mean().sqrt()) - 0.02) < 1e-15
    # solenoidal to rounding on a cubic grid (k . v = 0 with integer k)
    v, g = synthetic.evaluate(f, (12, 12, 12))
    assert float((g[0, 0] + g[1, 1] + g[2, 2]).abs().max()) < 1e-15


def test_fft_sampling_matches_direct_sum():
    f = synthetic.shell_field(3, 1, 3, 0.1)
    shape = (9, 10, 11)
    v, g = synthetic.evaluate(f, shape)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.integers(0, n, 20) for n in shape], axis=1)
    dv, dg = synthetic.evaluate_numpy(f, pts, shape, gradient=True)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    assert np.abs(dv - v[:, z, y, x].T.numpy()).max() < 1e-15
    assert np.abs(dg - g[:, :, z, y, x].permute(2, 0, 1).numpy()).max() < 1e-14


def test_seed_determinism():
    a = synthetic.shell_field(7, 1, 4, 0.02)
    b = synthetic.shell_field(7, 1, 4, 0.02)
    assert np.array_equal(a.v, b.v) and np.array_equal(a.k, b.k)
    assert not np.array_equal(a.v, synthetic.shell_field(8, 1, 4, 0.02).v)


def test_orszag_tang_fields_match_the_printed_formulas():
    """Sec. 4.4: u = U0 (-2 sin y, 2 sin x, 0), B = B0 (-2 sin 2y + sin z, 2 sin x + sin z,
    sin x + sin y) on a 2 pi box; checked against the formulas written with numpy's sin/cos at
    every node of a non-cubic grid, with the derivatives, mean squares and cross-helicity."""
    u0, b0 = 0.7, 0.8 * 0.7
    fu, fb = synthetic.orszag_tang(u0, b0)
    shape = (10, 12, 14)
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X, Y, Z = 2 * np.pi * x / nx, 2 * np.pi * y / ny, 2 * np.pi * z / nz
    qx, qy, qz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz
    u_ref = u0 * np.stack([-2 * np.sin(Y), 2 * np.sin(X), 0 * X])
    b_ref = b0 * np.stack([-2 * np.sin(2 * Y) + np.sin(Z), 2 * np.sin(X) + np.sin(Z), np.sin(X) + np.sin(Y)])
    zero = 0 * X
    du_ref = u0 * np.stack([  # [a, b] = d u_b / d x_a
        np.stack([zero, 2 * qx * np.cos(X), zero]),
        np.stack([-2 * qy * np.cos(Y), zero, zero]),
        np.stack([zero, zero, zero])])
    db_ref = b0 * np.stack([
        np.stack([zero, 2 * qx * np.cos(X), qx * np.cos(X)]),
        np.stack([-4 * qy * np.cos(2 * Y), zero, qy * np.cos(Y)]),
        np.stack([qz * np.cos(Z), qz * np.cos(Z), zero])])
    for f, ref, dref in ((fu, u_ref, du_ref), (fb, b_ref, db_ref)):
        v, g = synthetic.evaluate(f, shape)
        assert np.abs(v.numpy() - ref).max() < 1e-14
        assert np.abs(g.numpy() - dref).max() < 1e-14
        pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)[::37]
        assert np.abs(synthetic.evaluate_numpy(f, pts, shape) - ref.reshape(3, -1).T[::37]).max() < 1e-14
    assert abs(fu.mean_square - 4 * u0 ** 2) < 1e-15
    assert abs(fb.mean_square - 6 * b0 ** 2) < 1e-15
    assert abs((u_ref * b_ref).sum(0).mean() - 2 * u0 * b0) < 1e-15
    # solenoidal on any box: each component is independent of its own coordinate
    for dref in (du_ref, db_ref):
        assert np.abs(dref[0, 0] + dref[1, 1] + dref[2, 2]).max() == 0.0
