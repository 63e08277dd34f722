"""GPU adjoint (reverse mode through the C ABI) of a rollout of the step, for each way of
recomputing a checkpoint segment (moment route: trace lattices and saved states; stencil route:
saved states):
  * gradient of a magnetic-spectrum misfit w.r.t. the initial u and b against central finite
    differences of the same GPU forward (FP64 storage);
  * against torch autograd through the CPU oracle's rollout (definition route), FP64;
  * FP32 storage against FP64 (direction and size);
both J routes, forced, with checkpointed segments."""

import math

import pytest
import torch

import synthetic
from oracle import scheme

pytestmark = pytest.mark.gpu


def _fields(n, seed=0):
    u, _ = synthetic.evaluate(synthetic.shell_field(seed, 1, 2, 0.02), (n, n, n), gradient=False)
    b, _ = synthetic.evaluate(synthetic.shell_field(seed + 1, 1, 2, 0.02), (n, n, n), gradient=False)
    fu, _ = synthetic.evaluate(synthetic.shell_field(seed + 2, 0, 1, 1e-4, "radius"), (n, n, n), gradient=False)
    fb, _ = synthetic.evaluate(synthetic.shell_field(seed + 3, 0, 1, 1e-4, "radius"), (n, n, n), gradient=False)
    return u, b, fu, fb


ROUTES = ["moment-trace", "moment-state", "stencil-state"]


def _cfg(n, route, storage, steps, ckpt, fu, fb):
    from paper_2212_11024_amd.adjoint import RolloutConfig
    jmode, recompute = route.split("-")
    return RolloutConfig(n, n, n, 0.02, 0.03, 2.0, (0.01, -0.02, 0.04), storage, jmode, "aa", steps, ckpt, fu, fb,
                         recompute)


def _loss(B, target, nshells):
    from paper_2212_11024_amd.adjoint import spectrum_misfit
    return spectrum_misfit(B, target, nshells)


def _gpu_grad(u, b, cfg, target, nshells):
    from paper_2212_11024_amd.adjoint import rollout
    u0 = u.cuda().requires_grad_(True)
    b0 = b.cuda().requires_grad_(True)
    _, B = rollout(u0, b0, cfg)
    loss = _loss(B, target.cuda(), nshells)
    gu, gb = torch.autograd.grad(loss, (u0, b0))
    return float(loss), gu.cpu(), gb.cpu()


def _gpu_loss(u, b, cfg, target, nshells):
    from paper_2212_11024_amd.adjoint import rollout
    with torch.no_grad():
        _, B = rollout(u.cuda(), b.cuda(), cfg)
        return float(_loss(B, target.cuda(), nshells))


@pytest.mark.parametrize("route", ROUTES)
def test_adjoint_matches_central_differences(route):
    """16 seeded solenoidal directions (shells 1..5, unit rms), step 1e-4 of the field rms."""
    n, steps, ckpt, nshells = 12, 24, 8, 6
    print(f"[adjoint] FD {route}", flush=True)
    u, b, fu, fb = _fields(n)
    cfg = _cfg(n, route, "f64", steps, ckpt, fu, fb)
    target = torch.linspace(1e-5, 2e-6, nshells, dtype=torch.float64)
    loss, gu, gb = _gpu_grad(u, b, cfg, target, nshells)
    for j in range(16):
        du, _ = synthetic.evaluate(synthetic.shell_field(100 + j, 1, 5, 1.0), (n, n, n), gradient=False)
        db, _ = synthetic.evaluate(synthetic.shell_field(200 + j, 1, 5, 1.0), (n, n, n), gradient=False)
        eps = 1e-4 * 0.02
        lp = _gpu_loss(u + eps * du, b + eps * db, cfg, target, nshells)
        lm = _gpu_loss(u - eps * du, b - eps * db, cfg, target, nshells)
        fd = (lp - lm) / (2 * eps)
        ad = float((gu * du).sum() + (gb * db).sum())
        print(f"[adjoint] {route} direction {j}: adjoint {ad:.10e} fd {fd:.10e} rel {abs(ad - fd) / abs(fd):.2e}",
              flush=True)
        assert abs(ad - fd) <= 1e-6 * abs(fd)


def _oracle_grad(u, b, cfg, target, nshells):
    """Reference gradient: torch autograd through the oracle's rollout (T-matrix route)."""
    def sgrad(v):
        n = v.shape[-1]
        k = torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64)
        if n % 2 == 0:
            k[n // 2] = 0.0
        k = 2 * math.pi * k / n
        vh = torch.fft.fftn(v, dim=(1, 2, 3))
        return torch.stack([torch.fft.ifftn(1j * kk * vh, dim=(1, 2, 3)).real
                            for kk in (k.view(1, 1, n), k.view(1, n, 1), k.view(n, 1, 1))])

    def spectrum(B):
        n = B.shape[-1]
        f = torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64)
        sh = torch.floor(torch.sqrt(f.view(n, 1, 1) ** 2 + f.view(1, n, 1) ** 2 + f.view(1, 1, n) ** 2) + 0.5)
        sh = sh.long().reshape(-1)
        e = 0.5 * (torch.fft.fftn(B, dim=(1, 2, 3)).abs() ** 2).sum(0).reshape(-1) / n ** 6
        keep = sh < nshells
        return torch.zeros(nshells, dtype=torch.float64).index_add(0, sh[keep], e[keep])

    u0 = u.clone().requires_grad_(True)
    b0 = b.clone().requires_grad_(True)
    p = scheme.Params(cfg.nx, cfg.ny, cfg.nz, cfg.nu, cfg.eta, cfg.d_i, cfg.b0, cfg.jmode, "T",
                      cfg.force_u.double(), cfg.force_b.double())
    st = scheme.init_state(p, u0, b0, sgrad(u0), sgrad(b0))
    st = scheme.step(st, p, cfg.nsteps)
    _, _, B, _, _ = scheme.fields(st, p)
    e = spectrum(B)
    loss = ((e[1:] - target[1:]) ** 2).sum()
    return torch.autograd.grad(loss, (u0, b0))


@pytest.mark.parametrize("route", ROUTES)
def test_adjoint_matches_oracle_autograd(route):
    """16^3, 50 steps in checkpoint segments of 10, forced, both J routes."""
    n, steps, ckpt, nshells = 16, 50, 10, 8
    print(f"[adjoint] oracle {route}", flush=True)
    u, b, fu, fb = _fields(n, seed=3)
    cfg = _cfg(n, route, "f64", steps, ckpt, fu, fb)
    target = torch.linspace(1e-5, 2e-6, nshells, dtype=torch.float64)
    _, gu, gb = _gpu_grad(u, b, cfg, target, nshells)
    ou, ob = _oracle_grad(u, b, cfg, target, nshells)
    rel = float(torch.sqrt(((gu - ou) ** 2).sum() + ((gb - ob) ** 2).sum()) /
                torch.sqrt((ou ** 2).sum() + (ob ** 2).sum()))
    print(f"[adjoint] {route} GPU vs oracle autograd: relative {rel:.2e}", flush=True)
    assert rel < 1e-10


@pytest.mark.parametrize("route", ROUTES)
def test_fp32_adjoint_tracks_fp64(route):
    n, steps, ckpt, nshells = 12, 30, 10, 6
    u, b, fu, fb = _fields(n, seed=5)
    target = torch.linspace(1e-5, 2e-6, nshells, dtype=torch.float64)
    _, gu64, gb64 = _gpu_grad(u, b, _cfg(n, route, "f64", steps, ckpt, fu, fb), target, nshells)
    _, gu32, gb32 = _gpu_grad(u, b, _cfg(n, route, "f32", steps, ckpt, fu, fb), target, nshells)
    a = torch.cat([gu64.reshape(-1), gb64.reshape(-1)])
    c = torch.cat([gu32.reshape(-1), gb32.reshape(-1)])
    cos = float((a * c).sum() / (a.norm() * c.norm()))
    rel = float((a - c).norm() / a.norm())
    print(f"[adjoint] {route} FP32 vs FP64: cosine {cos:.6f}, relative {rel:.2e}", flush=True)
    assert cos > 0.999 and rel < 1e-3
