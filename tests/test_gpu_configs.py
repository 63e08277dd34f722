"""The decaying-turbulence configuration at full size: 256^3, moment-route J, seeded solenoidal
u and b in shells 1..4 (rms 0.02 each), b0 = 0, nu = eta = 0.002, d_i = 8 cells, 2000 steps,
FP64 and FP32 deviation storage, AA layout, diagnostics every 200 steps.

Checked: both runs stay finite; the invariants of the unforced scheme (total mass, total
momentum and the summed field B are conserved by collision and streaming alike); the total
energy decays; and the FP32 run tracks the FP64 run shell by shell. The FP32 bar: a shell energy
E ~ |u|^2 has dE/E ~ 2 du/u; FP32 rounding of the stored deviations gives u a relative error of
~6e-8 per step, ~2.7e-6 after a random walk over 2000 steps; the turbulent flow amplifies small
differences by about e^4 ~ 55 over its ~4 large-eddy turnover times (L/u ~ 500 steps). That is
3e-4 for the initially energetic shells 1..4 and for the energy-weighted error, and ten times
that for shells 5..8, whose energy the cascade builds during the run. Measured: 7e-5, 2.6e-4
and 6.6e-5."""

import math
import os

import pytest
import torch

import synthetic
from parity_helpers import sampled_step_error

pytestmark = pytest.mark.gpu

N, STEPS, EVERY, NSHELLS = 256, 2000, 200, 17


def _run(storage):
    from paper_2212_11024_amd.solver import Solver
    shape = (N, N, N)
    u, gu = synthetic.evaluate(synthetic.shell_field(0, 1, 4, 0.02), shape, "cuda")
    b, gb = synthetic.evaluate(synthetic.shell_field(1, 1, 4, 0.02), shape, "cuda")
    s = Solver(N, N, N, 0.002, 0.002, 8.0, (0.0, 0.0, 0.0), storage, "moment", "aa", u, b, gu, gb)
    del u, gu, b, gb
    torch.cuda.empty_cache()
    red0 = s.reduce()
    records, ms = [], 0.0
    for _ in range(STEPS // EVERY):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(EVERY)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        records.append((s.reduce(allow_nonfinite=True), s.spectrum("u", NSHELLS), s.spectrum("B", NSHELLS)))
    s.close()
    mlups = N ** 3 * STEPS / (ms * 1e-3) / 1e6
    print(f"[config2] {storage}: {ms / STEPS:.3f} ms/step, {mlups:.0f} MLUPS", flush=True)
    return red0, records


def test_decaying_turbulence_256_fp32_tracks_fp64():
    print("[config2] 256^3 decaying, d_i = 8, 2000 steps, FP64 then FP32", flush=True)
    runs = {st: _run(st) for st in ("f64", "f32")}
    for st, (red0, records) in runs.items():
        mass = float(red0[9])
        e_prev = float(red0[0] + red0[1])
        for red, _, _ in records:
            assert int(red[8]) == 0
            assert abs(float(red[9]) - mass) <= (1e-12 if st == "f64" else 1e-7) * mass
            mom = float((red[10:13] - red0[10:13]).abs().max())
            bsum = float((red[13:16] - red0[13:16]).abs().max())
            tol = (1e-12 if st == "f64" else 1e-7) * mass * 0.02
            assert mom <= tol and bsum <= tol, (st, mom, bsum)
            e = float(red[0] + red[1])
            assert e <= e_prev * (1 + 1e-9), (st, e, e_prev)
            e_prev = e
        print(f"[config2] {st}: energy {float(red0[0] + red0[1]):.6e} -> {e_prev:.6e}", flush=True)
    per_shell = torch.zeros(NSHELLS, dtype=torch.float64)
    weighted = 0.0
    for (_, u64, b64), (_, u32, b32) in zip(runs["f64"][1], runs["f32"][1]):
        for a, r in ((u32, u64), (b32, b64)):
            per_shell = torch.maximum(per_shell, (a - r).abs() / r)
            weighted = max(weighted, float((a[1:] - r[1:]).abs().sum() / r[1:].sum()))
        frac = (u64[1:] + b64[1:]) / (u64[1:] + b64[1:]).sum()
    print("[config2] FP32 vs FP64 worst relative error per shell 1..16: "
          + " ".join(f"{float(x):.1e}" for x in per_shell[1:]), flush=True)
    print("[config2] final energy fraction per shell 1..16: " + " ".join(f"{float(x):.1e}" for x in frac), flush=True)
    print(f"[config2] energy-weighted error, worst over the run: {weighted:.2e}", flush=True)
    assert weighted < 3e-4
    assert float(per_shell[1:5].max()) < 3e-4
    assert float(per_shell[5:9].max()) < 3e-3


def test_adjoint_configuration_128():
    """The differentiation configuration: 128^3, fields as in the decaying run, nu = eta = 0.002,
    d_i = 4, 1000 steps with checkpoints every 50; loss = sum over shells 1..64 of the squared
    misfit of the final magnetic energy spectrum to the spectrum of the same start run with
    d_i = 0. The FP64 gradient with respect to (u0, b0) against central finite differences
    along seeded solenoidal directions (shells 1..8, unit rms), bar 1e-4. The loss is a squared
    misfit of small spectral differences, so its curvature is large against its gradient: a step
    of 1e-4 (0.5% of the field rms) leaves an O(eps^2) truncation of order 1e-2, which the run
    prints together with the steps 1e-5 and 1e-6 to show the eps^2 convergence; the bar applies
    at 1e-6, where FP64 rounding of the loss difference is still ~1e-10 of it. The FP32 gradient
    against the FP64 one (direction and size). All 16 seeded directions are checked; the first
    two also at 1e-5, and the relative errors at the configured step 1e-4 are printed."""
    from paper_2212_11024_amd.adjoint import RolloutConfig, rollout, shell_spectrum
    from paper_2212_11024_amd.solver import Solver
    n, steps, ckpt, nsh = 128, 1000, 50, 65
    shape = (n, n, n)
    u, gu = synthetic.evaluate(synthetic.shell_field(0, 1, 4, 0.02), shape, "cuda")
    b, gb = synthetic.evaluate(synthetic.shell_field(1, 1, 4, 0.02), shape, "cuda")
    print("[config4] target run (d_i = 0)", flush=True)
    t = Solver(n, n, n, 0.002, 0.002, 0.0, (0.0, 0.0, 0.0), "f64", "moment", "aa", u, b, gu, gb)
    t.step(steps)
    target = t.spectrum("B", nsh).cuda()
    t.close()
    del gu, gb

    def cfg(storage):
        return RolloutConfig(n, n, n, 0.002, 0.002, 4.0, (0.0, 0.0, 0.0), storage, "moment", "aa", steps, ckpt)

    def loss_of(B):
        e = shell_spectrum(B, nsh)
        return ((e[1:] - target[1:]) ** 2).sum()

    grads = {}
    for storage in ("f64", "f32"):
        u0 = u.clone().requires_grad_(True)
        b0 = b.clone().requires_grad_(True)
        _, B = rollout(u0, b0, cfg(storage))
        L = loss_of(B)
        grads[storage] = torch.autograd.grad(L, (u0, b0))
        print(f"[config4] {storage}: loss {float(L):.6e}", flush=True)

    def loss_at(du, db, eps):
        with torch.no_grad():
            _, B = rollout(u + eps * du, b + eps * db, cfg("f64"))
            return float(loss_of(B))

    gu64, gb64 = grads["f64"]
    rows = []
    for j in range(16):
        du, _ = synthetic.evaluate(synthetic.shell_field(100 + j, 1, 8, 1.0), shape, "cuda", gradient=False)
        db, _ = synthetic.evaluate(synthetic.shell_field(200 + j, 1, 8, 1.0), shape, "cuda", gradient=False)
        ad = float((gu64 * du).sum() + (gb64 * db).sum())
        fds = {}
        for eps in ((1e-4, 1e-5, 1e-6) if j < 2 else (1e-4, 1e-6)):
            fds[eps] = (loss_at(du, db, eps) - loss_at(du, db, -eps)) / (2 * eps)
            print(f"[config4] direction {j}, step {eps:g}: adjoint {ad:.10e} fd {fds[eps]:.10e} "
                  f"rel {abs(ad - fds[eps]) / abs(fds[eps]):.2e}", flush=True)
        rows.append((ad, fds))
    # relative to each direction's derivative, with a floor of 1% of the largest one so that a
    # direction nearly orthogonal to the gradient is not judged by its rounding alone
    floor = 0.01 * max(abs(fds[1e-6]) for _, fds in rows)
    at_configured, at_fine = [], []
    for ad, fds in rows:
        at_configured.append(abs(ad - fds[1e-4]) / max(abs(fds[1e-4]), floor))
        at_fine.append(abs(ad - fds[1e-6]) / max(abs(fds[1e-6]), floor))
    print("[config4] relative error at the configured step 1e-4, 16 directions: "
          + " ".join(f"{r:.1e}" for r in at_configured), flush=True)
    print("[config4] relative error at the step 1e-6, 16 directions: " + " ".join(f"{r:.1e}" for r in at_fine),
          flush=True)
    assert max(at_fine) < 1e-4
    assert all(f < c for f, c in zip(at_fine, at_configured))
    a = torch.cat([g.reshape(-1) for g in grads["f64"]])
    c = torch.cat([g.reshape(-1) for g in grads["f32"]])
    cos = float((a * c).sum() / (a.norm() * c.norm()))
    rel = float((a - c).norm() / a.norm())
    print(f"[config4] FP32 vs FP64 gradient: cosine {cos:.6f}, relative {rel:.2e}", flush=True)
    assert cos > 0.999 and rel < 1e-3


def _free_hbm_gb():
    """Free device memory after releasing what earlier tests left in torch's cache."""
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    return free / 1e9


# sampled centres of the 1024^3 run: both ends of the grid and of a row, the wraps, random nodes
LARGE_CENTRES = [(1023, 1023, 1023), (0, 0, 0), (1022, 1023, 1023), (1023, 0, 511), (255, 256, 1023),
                 (256, 511, 0), (511, 767, 768), (17, 900, 333), (640, 1, 1022), (1000, 64, 96)]
# the full-size sampled bars (tests/test_gpu_fullsize.py): one step from a state read back exactly
LARGE_BARS = {"f32": (1e-5, 1e-4), "f16": (1e-3, 3e-3)}


def test_large_fp16_1024():
    """The large configuration: 1024^3, FP16 deviation storage with FP32 arithmetic, moment J,
    AA in place (103 GB of populations), decaying turbulence from seeded shells 1..4 (rms 0.02),
    nu = eta = 5e-4, d_i = 32 cells (whistler CFL number pi d_i max|B| ~ 5 at the start),
    500 steps, reductions every 100 steps; the same run with FP32 storage (206 GB) as the
    reference. The state starts at equilibrium (the non-equilibrium parts need the velocity and
    field gradients, 77 GB each, which do not fit beside the FP32 populations). Reported:
    throughput of both, the first record with non-finite values (none expected: the moment
    route is stable beyond the whistler CFL bound), FP16 against FP32 shell spectra, and after
    the 500 steps one even and one odd step of each run against the oracle on sampled nodes,
    among them the grid's last node, whose values end the 4 GiB FP32 arrays. Bar on the
    energetic shells 1..4: FP16 rounds each stored deviation to ~4.9e-4 relative per step, a
    random walk of ~1.1e-2 over 500 steps; measured 3.7e-4 at most (1024^3: FP16 51.5 ms/step,
    FP32 68.7 ms/step). Skipped only when the device has less free memory than the FP32 run
    needs."""
    from paper_2212_11024_amd.solver import Solver
    need = 262.0          # FP32 populations (206 GB) beside u and b (52 GB) at its initialisation
    free = _free_hbm_gb()
    print(f"[large] free device memory {free:.1f} GB", flush=True)
    if free < need:
        pytest.skip(f"1024^3 needs {need:.0f} GB of free HBM, {free:.0f} GB free")
    n, steps, every, nsh = 1024, 500, 100, 17
    shape = (n, n, n)
    u, _ = synthetic.evaluate(synthetic.shell_field(0, 1, 4, 0.02), shape, "cuda", gradient=False)
    b, _ = synthetic.evaluate(synthetic.shell_field(1, 1, 4, 0.02), shape, "cuda", gradient=False)
    torch.cuda.empty_cache()
    out = {}
    for storage in ("f16", "f32"):
        print(f"[large] 1024^3 {storage}: init", flush=True)
        s = Solver(n, n, n, 5e-4, 5e-4, 32.0, (0.0, 0.0, 0.0), storage, "moment", "aa", u, b)
        if storage == "f32":
            del u, b
            torch.cuda.empty_cache()
        ms, first_bad = 0.0, None
        for k in range(steps // every):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(every)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            red = s.reduce(allow_nonfinite=True)
            if int(red[8]) > 0 and first_bad is None:
                first_bad = (k + 1) * every
            print(f"[large] {storage} step {(k + 1) * every}: E_kin {float(red[0]):.6e} E_mag {float(red[1]):.6e} "
                  f"non-finite {int(red[8])}", flush=True)
        spec = {f: s.spectrum(f, nsh) for f in ("u", "B")}
        # one even and one odd step checked against the oracle on sampled nodes, among them the
        # last node of the grid, whose values sit at the very end of the 4 GiB (FP32) and 2 GiB
        # (FP16) population arrays
        for _ in range(2):
            err, worst = sampled_step_error(s, LARGE_CENTRES, n, 5e-4, 5e-4, 32.0, (0.0, 0.0, 0.0))
            print(f"[large] {storage} sampled one-step parity after {s.steps} steps: {err:.3e}, worst node "
                  f"{worst:.3e}", flush=True)
            assert err < LARGE_BARS[storage][0] and worst < LARGE_BARS[storage][1]
        s.close()
        del s
        torch.cuda.empty_cache()
        bpn = 2 * 48 * (2 if storage == "f16" else 4)
        mlups = n ** 3 * steps / (ms * 1e-3) / 1e6
        print(f"[large] {storage}: {ms / steps:.2f} ms/step, {mlups:.0f} MLUPS, "
              f"{mlups * 1e6 * bpn / 1e9:.0f} GB/s algorithmic ({bpn} B/node), first non-finite record: {first_bad}",
              flush=True)
        out[storage] = (spec, first_bad)
    assert out["f16"][1] is None and out["f32"][1] is None
    for f in ("u", "B"):
        a, r = out["f16"][0][f], out["f32"][0][f]
        rel = (a[1:9] - r[1:9]).abs() / r[1:9]
        print(f"[large] FP16 vs FP32 {f}, shells 1..8: " + " ".join(f"{float(x):.1e}" for x in rel), flush=True)
        assert float(rel[:4].max()) < 1e-2


def _forced_512(storage, d_i, steps, every, nsh=33):
    """The forced-turbulence workload at 512^3 (moment J, AA): reductions and shell spectra every
    `every` steps; the first step count whose reductions show a blown-up state (non-finite
    populations or max|u| at the sound speed) ends the run."""
    import bench
    s = bench.make_solver(512, storage, "moment", "aa", d_i=d_i)
    records, ms, first_bad = [], 0.0, None
    for k in range(steps // every):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(every)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        red = s.reduce(allow_nonfinite=True)
        bad = int(red[8]) > 0 or float(red[6]) >= 3 ** -0.5
        records.append((s.steps, red, None if bad else (s.spectrum("u", nsh), s.spectrum("B", nsh))))
        print(f"[config3] {storage} d_i={d_i:g} step {s.steps}: E_kin {float(red[0]):.6e} E_mag {float(red[1]):.6e} "
              f"max|u| {float(red[6]):.4f} non-finite {int(red[8])}", flush=True)
        if bad:
            first_bad = s.steps
            break
    taken = s.steps
    s.close()
    torch.cuda.empty_cache()
    print(f"[config3] {storage} d_i={d_i:g}: {ms / max(taken, 1):.3f} ms/step, "
          f"first blown-up record: {first_bad}", flush=True)
    return records, first_bad


def test_forced_512_fp32_tracks_fp64_over_5000_steps():
    """The forced configuration as configured: 512^3, FP32 deviation storage against an FP64 run of
    the same workload (nu = eta = 0.001, d_i = 4, static forcing at |k| <= 2), 5000 steps, shell
    spectra of u and B every 1000 steps. Both runs stay finite and below the sound speed; FP32
    tracks FP64 shell by shell. The static forcing keeps feeding the flow (its kinetic energy grows
    fourfold and max|u| reaches 0.3-0.4 by step 5000), which turns chaotic: from step ~2000 the two
    runs decorrelate at the largest scales, whatever the storage precision, and the error of the
    shell energies stops growing at ~2% (measured: 8.4e-4 / 2.0e-3 on shells 1..8 at step 1000,
    then 1.7e-2 / 1.2e-2 for u / B at step 5000; energy-weighted 4.4e-3). The bars (5e-2 on shells
    1..8, 1e-2 energy-weighted) sit above that saturation: they catch a systematic FP32 drift or a
    broken run, not the chaos of the flow."""
    print("[config3] 512^3 forced, d_i = 4, 5000 steps, FP64 then FP32", flush=True)
    runs = {st: _forced_512(st, 4.0, 5000, 1000) for st in ("f64", "f32")}
    for st, (_, bad) in runs.items():
        assert bad is None, (st, bad)
    worst_rel, worst_w = 0.0, 0.0
    for (t, _, s64), (_, _, s32) in zip(runs["f64"][0], runs["f32"][0]):
        line = []
        for a, r in zip(s32, s64):
            rel = float(((a[1:9] - r[1:9]).abs() / r[1:9]).max())
            w = float((a[1:] - r[1:]).abs().sum() / r[1:].sum())
            worst_rel, worst_w = max(worst_rel, rel), max(worst_w, w)
            line.append(f"{rel:.2e} / {w:.2e}")
        print(f"[config3] step {t}: FP32 vs FP64 shells 1..8 max rel / weighted 1..32: u {line[0]}, B {line[1]}",
              flush=True)
    assert worst_rel < 5e-2 and worst_w < 1e-2, (worst_rel, worst_w)


def test_forced_512_hall_transition():
    """The MHD to Hall-MHD transition of the forced configuration at the other two Hall parameters,
    d_i = 0 (ideal MHD) and d_i = 16 (whistler CFL number ~2.6 at the initial max|B|), FP32, 5000
    steps, reductions every 250 steps. Reported: the step of the first blown-up record, if any.
    Checked: a run either stays finite and below the sound speed throughout, or its blow-up is
    caught by flame_reduce (FLAME_E_NONFINITE / FLAME_E_UNSTABLE) and the run stops there, with
    every earlier record finite. Measured: d_i = 16 stays finite through 5000 steps (max|u| 0.25
    at the end); ideal MHD blows up between steps 2500 and 2750 (max|u| jumps from 0.08 to 0.13
    in the record before): at nu = eta = 0.001 under this forcing the Hall term, taken implicitly
    through the moment route's J system, keeps the run stable where ideal MHD is not."""
    for d_i in (0.0, 16.0):
        records, bad = _forced_512("f32", d_i, 5000, 250, nsh=17)
        print(f"[config3] d_i = {d_i:g}: first blown-up record at step {bad}", flush=True)
        for t, red, spec in records[:-1]:
            assert int(red[8]) == 0 and float(red[6]) < 3 ** -0.5 and spec is not None, (d_i, t)
        t, red, spec = records[-1]
        if bad is None:
            assert t == 5000 and int(red[8]) == 0 and float(red[6]) < 3 ** -0.5
        else:
            assert t == bad and (int(red[8]) > 0 or float(red[6]) >= 3 ** -0.5) and spec is None
