"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the same seeded
inputs. Error = relative L2 of the deviation populations (departures from the rest state)
over all 48 arrays. Bounds: FP64 storage 1e-12 against the extended-precision evaluation of
the oracle (the FP64 oracle's own rounding floor reaches a few 1e-12 after 100 steps, pinned in
test_oracle_extended.py); FP32 storage 1e-5 after 100 steps (FP32 rounding of O(100)
operations per step compounded over 100 steps, with a safety factor)."""

import math

import numpy as np
import pytest
import torch

import synthetic
from oracle import analytic, diagnostics, scheme

from oracle import extended

from parity_helpers import Case, deviation_error, extended_error, extended_run, gpu_solver, inputs, oracle_run

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}

CASES = {
    "ragged_moment": Case(13, 10, 9, jmode="moment"),
    "ragged_stencil": Case(13, 10, 9, jmode="stencil"),
    "hall_strong": Case(9, 8, 7, jmode="moment", d_i=8.0, seed=3),
    "forced": Case(12, 8, 8, jmode="stencil", forced=True, seed=5),
    "wide_x": Case(70, 5, 3, jmode="stencil", seed=7),
    # rows longer than one workgroup (256 nodes): the second block of each row is ragged
    "long_x": Case(257, 3, 3, jmode="moment", forced=True, seed=9),
    # the Orszag-Tang vortex of the paper's turbulence runs (Sec. 4.4, Sec. 5), ragged grid
    "orszag_tang": Case(13, 10, 9, jmode="moment", d_i=2.0, b0=(0.0, 0.0, 0.0), ic="orszag_tang"),
    # model variants: BGK fluid collision (S = omega I), electron MHD (Sec. 6), and both
    "bgk": Case(13, 10, 9, jmode="moment", forced=True, seed=23, collision="bgk"),
    "emhd": Case(13, 10, 9, jmode="moment", forced=True, seed=25, magnetic="emhd"),
    "bgk_emhd_stencil": Case(12, 8, 8, jmode="stencil", seed=27, collision="bgk", magnetic="emhd"),
}


def _print_case(name, **kw):
    print(f"[gpu parity] {name} {kw}", flush=True)


@pytest.mark.parametrize("layout", ["ab", "aa"])
@pytest.mark.parametrize("name", list(CASES))
def test_initial_state(name, layout):
    case = CASES[name]
    _print_case(name, layout=layout, step=0)
    s = gpu_solver(case, "f64", layout)
    assert extended_error(s, extended_run(case, 0)) < 1e-15
    p, st = oracle_run(case, 0)
    assert deviation_error(s, p, st) < 1e-14


@pytest.mark.parametrize("layout", ["ab", "aa"])
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_step_parity(name, layout):
    case = CASES[name]
    steps = 21   # odd: ends on the swapped AA slots
    _print_case(name, layout=layout, storage="f64", steps=steps)
    s = gpu_solver(case, "f64", layout)
    s.step(steps)
    assert extended_error(s, extended_run(case, steps)) < TOL["f64"]


@pytest.mark.parametrize("ic", ["shell", "orszag_tang"])
@pytest.mark.parametrize("jmode", ["moment", "stencil"])
def test_fp64_parity_100_steps(jmode, ic):
    # 100 steps: within 1e-12 of the extended evaluation, and within the FP64 oracle's own
    # floor of its literal T-matrix route
    case = Case(8, 7, 6, jmode=jmode, seed=11, ic=ic)
    _print_case("100 steps", jmode=jmode, ic=ic)
    s = gpu_solver(case, "f64", "aa")
    s.step(100)
    err = extended_error(s, extended_run(case, 100))
    print("FP64 error vs extended after 100 steps:", err)
    assert err < TOL["f64"]
    p, st = oracle_run(case, 100, route="T")
    assert deviation_error(s, p, st) < 2e-11


@pytest.mark.parametrize("layout", ["ab", "aa"])
@pytest.mark.parametrize("name", ["ragged_moment", "ragged_stencil", "forced", "orszag_tang", "bgk", "emhd",
                                  "bgk_emhd_stencil"])
def test_fp32_step_parity_100_steps(name, layout):
    case = CASES[name]
    _print_case(name, layout=layout, storage="f32", steps=100)
    p, st = oracle_run(case, 100, ftype=torch.float32)
    s = gpu_solver(case, "f32", layout)
    s.step(100)
    assert deviation_error(s, p, st) < TOL["f32"]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("jmode", ["moment", "stencil"])
def test_aa_equals_ab_bitwise(storage, jmode):
    case = Case(11, 9, 8, jmode=jmode, seed=2)
    _print_case("aa-vs-ab", storage=storage, jmode=jmode)
    a = gpu_solver(case, storage, "aa")
    b = gpu_solver(case, storage, "ab")
    for n in (1, 4, 7):
        a.step(n)
        b.step(n)
        fa, ga = a.get_populations()
        fb, gb = b.get_populations()
        assert torch.equal(fa, fb) and torch.equal(ga, gb)


def test_run_to_run_determinism():
    case = CASES["ragged_stencil"]
    _print_case("determinism")
    a = gpu_solver(case, "f32", "aa")
    b = gpu_solver(case, "f32", "aa")
    a.step(30)
    b.step(30)
    assert torch.equal(a.get_populations()[0], b.get_populations()[0])
    assert torch.equal(a.reduce(), b.reduce())


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_launch_shape_independence(storage, monkeypatch):
    """The state does not depend on the launch shape, bit for bit: the planes per workgroup of the
    curl-stencil kernel (FLAME_ZCHUNK_PLANES: the built-in 32, 5 with a ragged last chunk, 1, the
    whole column and more than it) and the threads per row block of the node-local kernels
    (FLAME_ROW_THREADS: one block per row, or 64, 128 and 192 threads, so that a 257-node row
    spans several blocks with a ragged last one; 512 is taken as the kernels' launch bound of
    256), and the addressing of the node-local step
    (FLAME_GLOBAL_ADDRESSING: buffer resources or 64-bit global addresses), on forced runs over 7
    steps (both AA parities)."""
    cases = [(Case(13, 10, 37, jmode="stencil", forced=True, seed=61), "FLAME_ZCHUNK_PLANES", ["0", "5", "1", "37", "64"]),
             (Case(257, 3, 4, jmode="moment", forced=True, seed=63), "FLAME_ROW_THREADS", ["0", "64", "128", "192", "512"]),
             (Case(33, 17, 9, jmode="moment", forced=True, seed=65), "FLAME_GLOBAL_ADDRESSING", ["0", "1"])]
    for case, var, values in cases:
        ref = None
        for v in values:
            monkeypatch.setenv(var, v)
            _print_case("launch shape", storage=storage, jmode=case.jmode, **{var: v})
            s = gpu_solver(case, storage, "aa")
            s.step(7)
            f, g = s.get_populations(deviations=True)
            s.close()
            if ref is None:
                ref = (f, g)
            else:
                assert torch.equal(f, ref[0]) and torch.equal(g, ref[1]), (var, v)
        monkeypatch.delenv(var)


@pytest.mark.parametrize("shape", [(13, 10, 9), (48, 40, 36)])
def test_spectra_are_bitwise_reproducible(shape):
    """Shell spectra, dissipation spectra and the energy-transfer terms sum in a fixed order (no
    atomics): two runs from the same inputs, and two calls on one state, agree bit for bit. The
    larger grid spreads the half spectrum over many binning blocks and puts many lanes of a
    wavefront into one shell."""
    case = Case(*shape, jmode="stencil", forced=True, seed=31, kmax=3)
    _print_case("spectra determinism", shape=shape)
    runs = []
    for _ in range(2):
        s = gpu_solver(case, "f64", "aa")
        s.step(5)
        ns = max(shape) // 2 + 1
        out = [s.spectrum("u", ns), s.spectrum("B", ns), s.dissipation_spectrum("u", ns),
               s.dissipation_spectrum("B", ns), s.energy_transfer(ns, hall=True)]
        again = [s.spectrum("u", ns), s.spectrum("B", ns), s.dissipation_spectrum("u", ns),
                 s.dissipation_spectrum("B", ns), s.energy_transfer(ns, hall=True)]
        for x, y in zip(out, again):
            assert torch.equal(x, y)
        runs.append(out)
        s.close()
    for x, y in zip(*runs):
        assert torch.equal(x, y)
        assert bool(torch.isfinite(x).all())


def test_unstable_state_is_reported():
    """flame_reduce returns FLAME_E_UNSTABLE (after filling its slots) once max |u| reaches the
    lattice sound speed 1/sqrt(3), and FLAME_OK below it. The states are set from the host: mass
    moved from the rest population to the +x one gives a uniform flow u_x = m at rho = 1."""
    from paper_2212_11024_amd import _lib as L
    case = CASES["ragged_moment"]
    s = gpu_solver(case, "f64", "aa")
    rest_f, rest_g = s.rest_populations()
    shape = (case.nz, case.ny, case.nx)
    plus_x = 14                          # c = (1, 0, 0) in the App. A order
    for m, expect in ((0.5, L.FLAME_OK), (0.7, L.FLAME_E_UNSTABLE)):
        f = rest_f.view(27, 1, 1, 1).expand(27, *shape).clone()
        f[0] -= m
        f[plus_x] += m
        g = rest_g.view(7, 3, 1, 1, 1).expand(7, 3, *shape).clone()
        s.set_populations(f, g)
        code, vals = L.flame_reduce(s.ctx, allow_nonfinite=True)
        assert code == expect, (m, code, L.flame_last_error(s.ctx))
        assert abs(vals[6] - m) < 1e-12 and vals[8] == 0
        if expect != L.FLAME_OK:
            with pytest.raises(L.FlameError) as e:
                s.reduce()
            assert e.value.code == L.FLAME_E_UNSTABLE
    s.close()


def test_whistler_cfl_warning():
    """flame_init returns the warning FLAME_W_CFL (and a usable context) when the advisory whistler
    number pi d_i max|B| of the initial field exceeds 1, FLAME_OK otherwise (Sec. 3.4)."""
    from paper_2212_11024_amd import _lib as L
    for d_i, expect in ((0.5, L.FLAME_OK), (8.0, L.FLAME_W_CFL)):
        case = Case(9, 8, 7, jmode="moment", d_i=d_i, b0=(0.0, 0.0, 0.1), seed=17)
        s = gpu_solver(case, "f32", "aa")
        _, _, b, _, _, _ = inputs(case)
        bmax = float(((b + torch.tensor(case.b0, dtype=b.dtype).view(3, 1, 1, 1)) ** 2).sum(0).sqrt().max())
        assert abs(s.cfl - math.pi * d_i * bmax) <= 1e-12 * s.cfl
        assert s.status == expect, (d_i, s.cfl, s.status)
        s.step(3)
        assert int(s.reduce()[8]) == 0
        s.close()


def test_set_get_roundtrip_and_resume():
    case = CASES["ragged_moment"]
    _print_case("resume")
    for storage in ("f64", "f32", "f16"):
        a = gpu_solver(case, storage, "aa")
        a.step(5)
        f, g = a.get_populations(deviations=True)
        b = gpu_solver(case, storage, "aa")
        b.set_populations(f, g, deviations=True)
        fb, gb = b.get_populations(deviations=True)
        assert torch.equal(f, fb) and torch.equal(g, gb)
        a.step(6)
        b.step(6)
        assert torch.equal(a.get_populations(True)[0], b.get_populations(True)[0])
        # full values round-trip to within the rounding of the rest-plus-deviation sum
        ff, gf = a.get_populations()
        b.set_populations(ff, gf)
        assert (b.get_populations()[0] - ff).abs().max() < 1e-15


def test_fields_reductions_spectra_vs_oracle():
    for jmode in ("moment", "stencil"):
        case = Case(12, 12, 12, jmode=jmode, forced=True, seed=13)
        _print_case("diagnostics", jmode=jmode)
        p, st = oracle_run(case, 9)
        s = gpu_solver(case, "f64", "aa")
        s.step(9)
        rho, u, B, J, d = [t.cpu() for t in s.fields()]
        orho, ou, oB, oJ, od = scheme.fields(st, p)
        for a, b in ((rho, orho), (u, ou), (B, oB), (J, oJ), (d, od)):
            assert (a - b).abs().max() <= 1e-12 * max(1e-3, float(b.abs().max()))
        r = s.reduce()
        ro = diagnostics.reductions(st, p)
        assert torch.allclose(r[:10], ro[:10], rtol=1e-11, atol=1e-18)
        # sums over the grid: absolute agreement relative to the total mass
        assert (r[10:] - ro[10:]).abs().max() < 1e-12 * float(ro[9])
        ns = diagnostics.max_shell(p.shape)
        for field, ref in (("u", ou), ("B", oB)):
            e = s.spectrum(field, ns)
            eo = torch.tensor(diagnostics.spectrum(ref, ns))
            assert torch.allclose(e, eo, rtol=1e-10, atol=1e-20 + 1e-12 * float(eo.max()))


@pytest.mark.parametrize("shape", [(13, 10, 9), (12, 10, 8), (32, 32, 32)])
def test_dissipation_spectrum_vs_oracle(shape):
    """k^2-weighted shell spectra on odd, even (Nyquist planes) and cubic grids. On 32^3 also
    their sum for B against the GPU's own <|J|^2> from the moments: the moment route's J is the
    curl of B only up to the scheme's truncation error, O((k dx)^2) with k up to 2 (2 pi / 32),
    here 0.2% (16^3 gives 7%), so that comparison takes a 1% bound."""
    case = Case(*shape, jmode="moment", d_i=1.0, ic="orszag_tang", b0=(0.0, 0.0, 0.0), seed=17)
    _print_case("dissipation spectrum", shape=shape)
    p, st = oracle_run(case, 5)
    s = gpu_solver(case, "f64", "aa")
    s.step(5)
    _, ou, oB, _, _ = scheme.fields(st, p)
    ns = diagnostics.max_shell(p.shape)
    for field, ref in (("u", ou), ("B", oB)):
        d = s.dissipation_spectrum(field, ns)
        do = torch.tensor(diagnostics.dissipation_spectrum(ref, ns))
        assert torch.allclose(d, do, rtol=1e-10, atol=1e-20 + 1e-12 * float(do.max()))
    if shape == (32, 32, 32):
        J = s.fields()[3]
        j2 = float((J * J).sum(0).mean())
        assert abs(float(s.dissipation_spectrum("B", ns).sum()) - j2) < 0.01 * j2


@pytest.mark.parametrize("jmode", ["moment", "stencil"])
@pytest.mark.parametrize("shape", [(13, 10, 9), (12, 10, 8), (16, 16, 16)])
def test_energy_transfer_vs_oracle(shape, jmode):
    """The three transfer terms per shell against the oracle's, computed from the oracle's own
    node fields after 7 steps (odd: swapped AA slots), on odd, even (Nyquist planes) and cubic
    grids, for both J routes; b0 != 0 puts the mean field into the induction term."""
    case = Case(*shape, jmode=jmode, d_i=1.5, ic="orszag_tang", b0=(0.01, -0.02, 0.03), seed=19)
    _print_case("energy transfer", shape=shape, jmode=jmode)
    p, st = oracle_run(case, 7)
    s = gpu_solver(case, "f64", "aa")
    s.step(7)
    _, ou, oB, oJ, _ = scheme.fields(st, p)
    ns = diagnostics.max_shell(p.shape)
    got = s.energy_transfer(ns, hall=True)
    ref = torch.tensor(np.stack(diagnostics.energy_transfer(ou, oB, oJ, ns, d_i=case.d_i)))
    scale = float(ref.abs().max())
    assert scale > 0 and float(ref[3].abs().max()) > 0
    assert float((got - ref).abs().max()) < 1e-11 * scale
    # without the Hall row the three terms are the same (up to the order of the shell sums)
    assert float((s.energy_transfer(ns) - got[:3]).abs().max()) < 1e-13 * scale


def test_exact_wave_on_gpu_matches_oracle():
    # the analytic Hall wave (32^3, FP64, 200 steps): GPU vs the oracle's z-column, which is
    # exact for a z-wave by translation invariance
    N, amp, b0, d_i, nu = 32, 1e-3, 0.1, 2.0, 0.01
    for jmode in ("moment", "stencil"):
        _print_case("wave", jmode=jmode)
        k = 2 * math.pi / N
        be = analytic.beta(d_i, k, +1)
        uf = synthetic.wave_field(amp)
        p1 = scheme.Params(1, 1, N, nu, nu, d_i, (0.0, 0.0, b0), jmode, "closed")
        u1, gu1 = synthetic.evaluate(uf, (1, 1, N))
        b1, gb1 = synthetic.evaluate(synthetic.scaled(uf, be), (1, 1, N))
        xp = extended.Params(p1)
        xf, xg = extended.init_state(xp, u1, b1, gu1, gb1)
        xf, xg = extended.step(xf, xg, xp, 200)
        fr, gr = extended.rest_state(xp, (N, 1, 1))
        ref = (np.broadcast_to(xf - fr, (27, N, N, N)), np.broadcast_to(xg - gr, (7, 3, N, N, N)))
        from paper_2212_11024_amd.solver import Solver
        u, gu = synthetic.evaluate(uf, (N, N, N))
        b, gb = synthetic.evaluate(synthetic.scaled(uf, be), (N, N, N))
        s = Solver(N, N, N, nu, nu, d_i, (0.0, 0.0, b0), "f64", jmode, "aa", u, b, gu, gb)
        s.step(200)
        assert extended_error(s, ref) < TOL["f64"]
        # and the analytic solution itself
        _, U, Bf, _, _ = [t.cpu() for t in s.fields()]
        ue, bexact = analytic.wave(N, 200, amp, b0, nu, d_i, +1)
        err = torch.linalg.norm(U[:, :, 0, 0] - ue) / torch.linalg.norm(ue)
        assert float(err) < (0.01 if jmode == "stencil" else 0.05)


def test_degenerate_grids():
    # single-node cross-sections (moment route) and the smallest stencil grid
    for case in (Case(1, 1, 16, jmode="moment", kmax=0), Case(3, 3, 3, jmode="stencil")):
        _print_case("degenerate", shape=case.shape)
        if case.nx == 1:
            uf = synthetic.wave_field(1e-3, kz=2)
            u, gu = synthetic.evaluate(uf, case.shape)
            p = scheme.Params(1, 1, case.nz, case.nu, case.eta, case.d_i, case.b0, case.jmode, "closed")
            xp = extended.Params(p)
            xf, xg = extended.init_state(xp, u, 0.5 * u, gu, 0.5 * gu)
            xf, xg = extended.step(xf, xg, xp, 13)
            fr, gr = extended.rest_state(xp, xf.shape[1:])
            from paper_2212_11024_amd.solver import Solver
            s = Solver(1, 1, case.nz, case.nu, case.eta, case.d_i, case.b0, "f64", "moment", "aa", u, 0.5 * u, gu,
                       0.5 * gu)
            s.step(13)
            assert extended_error(s, (xf - fr, xg - gr)) < TOL["f64"]
        else:
            s = gpu_solver(case, "f64", "aa")
            s.step(13)
            assert extended_error(s, extended_run(case, 13)) < TOL["f64"]
    # zero steps leave the state unchanged
    s = gpu_solver(CASES["ragged_moment"], "f32", "aa")
    f0 = s.get_populations()[0].clone()
    s.step(0)
    assert torch.equal(f0, s.get_populations()[0])


def _axis_limited_field(shape, seed, amp, nmodes=4):
    """A few random Fourier modes with |k_a| <= (n_a - 1) / 2 on every axis (no aliasing, no
    Nyquist content), for grids too thin for the shell fields."""
    import itertools
    lim = [(n - 1) // 2 for n in shape]
    ks = [k for k in itertools.product(*(range(-m, m + 1) for m in lim))
          if k[2] > 0 or (k[2] == 0 and (k[1] > 0 or (k[1] == 0 and k[0] > 0)))]
    rng = np.random.default_rng(seed)
    ks = [ks[i] for i in rng.permutation(len(ks))[:nmodes]]
    v = amp * (rng.standard_normal((len(ks), 3)) + 1j * rng.standard_normal((len(ks), 3)))
    return synthetic.ModeField(np.array(ks, dtype=np.int64).reshape(-1, 3), v)


@pytest.mark.parametrize("shape", [(1, 12, 10), (1, 1, 16), (2, 3, 4), (5, 1, 6)])
def test_spectral_diagnostics_on_degenerate_grids(shape):
    """Energy spectra, dissipation spectra and transfer terms on one-node-thick axes and on the
    smallest grids (length-2 and length-4 axes carry a Nyquist plane) against the oracle."""
    from paper_2212_11024_amd.solver import Solver
    _print_case("degenerate diagnostics", shape=shape)
    u, gu = synthetic.evaluate(_axis_limited_field(shape, 41, 0.01), shape)
    b, gb = synthetic.evaluate(_axis_limited_field(shape, 43, 0.01), shape)
    nx, ny, nz = shape
    p = scheme.Params(nx, ny, nz, 0.02, 0.03, 1.0, (0.01, 0.0, 0.02), "moment", "closed")
    st = scheme.step(scheme.init_state(p, u, b, gu, gb), p, 3)
    s = Solver(nx, ny, nz, p.nu, p.eta, p.d_i, p.b0, "f64", "moment", "aa", u, b, gu, gb)
    s.step(3)
    _, ou, oB, oJ, _ = scheme.fields(st, p)
    ns = diagnostics.max_shell(p.shape)
    for field, ref in (("u", ou), ("B", oB)):
        e, eo = s.spectrum(field, ns), torch.tensor(diagnostics.spectrum(ref, ns))
        d, do = s.dissipation_spectrum(field, ns), torch.tensor(diagnostics.dissipation_spectrum(ref, ns))
        assert torch.allclose(e, eo, rtol=1e-10, atol=1e-20 + 1e-12 * float(eo.abs().max()))
        assert torch.allclose(d, do, rtol=1e-10, atol=1e-20 + 1e-12 * float(do.abs().max()))
    got = s.energy_transfer(ns)
    ref = torch.tensor(np.stack(diagnostics.energy_transfer(ou, oB, oJ, ns)))
    assert float((got - ref).abs().max()) <= 1e-11 * max(float(ref.abs().max()), 1e-30)
    s.close()


def test_diagnostic_argument_errors():
    """Host-side refusals of the spectral diagnostics: no kernel is launched by these calls."""
    from paper_2212_11024_amd import _lib as L
    s = gpu_solver(Case(8, 6, 5, jmode="moment"), "f64", "aa")
    import ctypes
    buf = (ctypes.c_double * 8)()
    lib = L.load()
    assert lib.flame_dissipation_spectrum(s.ctx, 2, 8, buf) == L.FLAME_E_INVAL
    assert lib.flame_dissipation_spectrum(s.ctx, 0, 0, buf) == L.FLAME_E_INVAL
    assert lib.flame_dissipation_spectrum(s.ctx, 0, 8, None) == L.FLAME_E_INVAL
    assert lib.flame_energy_transfer(s.ctx, 0, buf, buf, buf, None) == L.FLAME_E_INVAL
    assert lib.flame_energy_transfer(s.ctx, 5000, buf, buf, buf, buf) == L.FLAME_E_INVAL
    assert lib.flame_energy_transfer(s.ctx, 8, buf, None, buf, None) == L.FLAME_E_INVAL
    assert lib.flame_energy_transfer(None, 8, buf, buf, buf, None) == L.FLAME_E_INVAL
    s.close()


def test_nonfinite_detection():
    case = CASES["ragged_moment"]
    s = gpu_solver(case, "f32", "aa")
    f, g = s.get_populations()
    f = f.clone()
    f[3, 2, 1, 4] = float("nan")
    s.set_populations(f, g)
    r = s.reduce(allow_nonfinite=True)
    assert r[8] == 1
    from paper_2212_11024_amd._lib import FlameError
    with pytest.raises(FlameError):
        s.reduce()


@pytest.mark.parametrize("model", [{}, {"collision": "bgk"}, {"magnetic": "emhd", "jmode": "moment"}])
def test_fp16_storage_tracks_fp32(model):
    case = Case(12, 10, 9, **{"jmode": "stencil", "seed": 4, **model})
    _print_case("f16", steps=50, **model)
    ref = extended_run(case, 50)
    a = gpu_solver(case, "f16", "aa")
    a.step(50)
    err = extended_error(a, ref)
    b = gpu_solver(case, "f32", "aa")
    b.step(50)
    print("deviation error after 50 steps: f16", err, "f32", extended_error(b, ref), flush=True)
    assert err < 5e-3


@pytest.mark.parametrize("jmode", ["moment", "stencil"])
def test_initial_state_from_central_differences(jmode):
    # no gradients passed, non-equilibrium initialisation on: the library takes central
    # differences of u and b on the grid, which the oracle receives explicitly
    from paper_2212_11024_amd.solver import Solver
    case = Case(11, 9, 7, jmode=jmode, forced=True, seed=21)
    _print_case("central-difference init", jmode=jmode)
    u, gu, b, gb, fu, fb = inputs(case)
    s = Solver(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, "f64", jmode, "aa",
               u, b, None, None, fu, fb, init_noneq=True)
    p = scheme.Params(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, jmode, "closed", fu, fb)
    st = scheme.init_state(p, u, b, scheme.central_gradient(u), scheme.central_gradient(b))
    assert deviation_error(s, p, st) < 1e-14
    s.step(5)
    assert deviation_error(s, p, scheme.step(st, p, 5)) < 1e-13


def _gpu_from(case, u, gu, b, gb, storage="f64"):
    from paper_2212_11024_amd.solver import Solver
    return Solver(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, storage, case.jmode, "aa",
                  u, b, gu, gb)


@pytest.mark.parametrize("jmode", ["moment", "stencil"])
def test_ideal_mhd_limit(jmode):
    # d_i = 0: no Hall term (the moment-route solve reduces to the ideal one, the stencil J is unused)
    case = Case(9, 8, 7, jmode=jmode, d_i=0.0, seed=31)
    _print_case("ideal MHD", jmode=jmode)
    s = gpu_solver(case, "f64", "aa")
    s.step(21)
    assert extended_error(s, extended_run(case, 21)) < TOL["f64"]


def test_field_free_flow_stays_field_free():
    # b = 0 and b0 = 0: pure hydrodynamics; the magnetic populations stay exactly at rest
    case = Case(10, 9, 8, jmode="moment", b0=(0.0, 0.0, 0.0), seed=33)
    _print_case("field-free")
    u, gu, b, gb, _, _ = inputs(case)
    b, gb = torch.zeros_like(b), torch.zeros_like(gb)
    s = _gpu_from(case, u, gu, b, gb)
    p = scheme.Params(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, "moment", "closed")
    st = scheme.step(scheme.init_state(p, u, b, gu, gb), p, 21)
    s.step(21)
    assert deviation_error(s, p, st) < 1e-12
    _, g = s.get_populations(deviations=True)
    assert int(torch.count_nonzero(g)) == 0


def test_one_node_thick_grid():
    # nx = 1 (a periodic 2-D flow in y, z): every x-shift wraps onto the node itself
    case = Case(1, 12, 10, jmode="moment", seed=35)
    _print_case("nx = 1")
    ny, nz = case.ny, case.nz
    y = torch.arange(ny, dtype=torch.float64).view(1, ny, 1).expand(nz, ny, 1)
    z = torch.arange(nz, dtype=torch.float64).view(nz, 1, 1).expand(nz, ny, 1)
    ky, kz = 2 * math.pi / ny, 2 * math.pi / nz
    A = 0.02
    # solenoidal: each component is independent of its own coordinate
    u = torch.stack([A * torch.sin(ky * y + kz * z), A * torch.cos(kz * z), A * torch.sin(ky * y)])
    b = torch.stack([A * torch.cos(kz * z), A * torch.sin(2 * kz * z), A * torch.cos(ky * y)])
    gu = torch.zeros(3, 3, nz, ny, 1, dtype=torch.float64)
    gb = torch.zeros_like(gu)
    gu[1, 0] = A * ky * torch.cos(ky * y + kz * z)
    gu[2, 0] = A * kz * torch.cos(ky * y + kz * z)
    gu[2, 1] = -A * kz * torch.sin(kz * z)
    gu[1, 2] = A * ky * torch.cos(ky * y)
    gb[2, 0] = -A * kz * torch.sin(kz * z)
    gb[2, 1] = 2 * A * kz * torch.cos(2 * kz * z)
    gb[1, 2] = -A * ky * torch.sin(ky * y)
    s = _gpu_from(case, u, gu, b, gb)
    p = scheme.Params(case.nx, ny, nz, case.nu, case.eta, case.d_i, case.b0, "moment", "closed")
    st = scheme.step(scheme.init_state(p, u, b, gu, gb), p, 21)
    s.step(21)
    assert deviation_error(s, p, st) < 1e-12


@pytest.mark.parametrize("name", ["bgk", "emhd", "bgk_emhd_stencil"])
def test_variant_fp64_parity_100_steps(name):
    # the model variants over 100 steps against the extended evaluation of the oracle
    case = CASES[name]
    _print_case(name, storage="f64", steps=100)
    s = gpu_solver(case, "f64", "aa")
    s.step(100)
    assert extended_error(s, extended_run(case, 100)) < TOL["f64"]


def test_reverse_mode_refuses_model_variants():
    """Host-side refusals: the state-saving step, the adjoint entry points and the trace calls
    are built for the paper's model only."""
    from paper_2212_11024_amd import _lib as L
    for kw in ({"collision": "bgk"}, {"magnetic": "emhd"}):
        case = Case(8, 6, 5, jmode="moment", **kw)
        s = gpu_solver(case, "f32", "aa")
        buf = torch.empty(51 * s.n * 4, dtype=torch.uint8, device=s.device)
        lat = torch.empty((2, L.flame_trace_bytes(s.ctx)), dtype=torch.uint8, device=s.device)
        calls = (lambda: L.flame_step_save(s.ctx, buf.data_ptr()),
                 lambda: L.flame_trace_export(s.ctx, lat[0].data_ptr()),
                 lambda: L.flame_trace_step(s.ctx, lat[0].data_ptr(), lat[1].data_ptr()))
        for call in calls:
            with pytest.raises(L.FlameError) as e:
                call()
            assert e.value.code == L.FLAME_E_UNSUPPORTED
        s.close()


def test_placement_probe_keeps_results():
    """Choosing the population buffer by timing trial steps on candidates changes nothing in the
    run: the kept buffer is re-initialised, and the state after some steps is bitwise that of a
    run without the probe."""
    from paper_2212_11024_amd.solver import Solver
    case = Case(24, 20, 16, jmode="moment", forced=True, seed=29)
    _print_case("placement probe", trials=3)
    u, gu, b, gb, fu, fb = inputs(case)
    runs = []
    for trials in (1, 3):
        s = Solver(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, "f32", "moment", "aa",
                   u, b, gu, gb, fu, fb, placement_trials=trials)
        assert (s.placement_ms is None) if trials == 1 else (len(s.placement_ms) == 3)
        s.step(9)
        runs.append(s.get_populations())
        s.close()
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])

