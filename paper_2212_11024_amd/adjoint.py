"""Gradients of a rollout of the Hall-MHD step with respect to its initial fields.

``FlameRollout`` is a ``torch.autograd.Function``: forward initialises a run from (u0, b0,
grad u0, grad b0) and advances it ``nsteps`` steps, returning the final node fields (u_T, B_T);
backward runs the library's hand-written adjoint. Memory is bounded by checkpointing every
``ckpt`` steps, and the backward recomputes one segment at a time:
  * trace recompute (moment route, AA layout): checkpoints are exact trace lattices
    (``flame_trace_export``); a segment is recomputed as a chain of trace lattices
    (``flame_trace_step``, one ordinary step each) and swept back with
    ``flame_adjoint_trace_step``, which pulls each step's state from the chain;
  * state recompute (any route): checkpoints are the exact deviation state; a segment is
    recomputed with ``flame_step_save``, which also records each step's pre-collision state and
    J, and swept back with ``flame_adjoint_step``.
Then the adjoint of the initial state is applied. All arithmetic is in libflame.so; this module
moves pointers.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

from . import _lib as L
from .solver import Solver


def spectral_gradient(v: torch.Tensor) -> torch.Tensor:
    """grad[a, c] = d v_c / d x_a of a periodic field v (3, nz, ny, nx), by FFT (differentiable).

    Exact for fields whose modes lie below the Nyquist wavenumber on every axis."""
    nz, ny, nx = v.shape[1:]
    dev, dt = v.device, v.dtype

    def k(n):
        f = torch.fft.fftfreq(n, d=1.0 / n, device=dev, dtype=dt)
        if n % 2 == 0:
            f[n // 2] = 0.0           # the Nyquist mode has no well-defined derivative
        return 2.0 * math.pi * f / n

    kx = k(nx).view(1, 1, nx)
    ky = k(ny).view(1, ny, 1)
    kz = k(nz).view(nz, 1, 1)
    vh = torch.fft.fftn(v, dim=(1, 2, 3))
    out = []
    for ka in (kx, ky, kz):
        out.append(torch.fft.ifftn(1j * ka * vh, dim=(1, 2, 3)).real)
    return torch.stack(out)


def shell_spectrum(v: torch.Tensor, nshells: int) -> torch.Tensor:
    """E(s) = 1/2 sum_{round(|k|) = s} |v_hat|^2, v_hat = DFT(v) / ncell, shells 0..nshells-1
    (differentiable torch version of the library's flame_spectrum)."""
    nz, ny, nx = v.shape[1:]
    n = nx * ny * nz
    dev = v.device
    fz = torch.fft.fftfreq(nz, d=1.0 / nz, device=dev, dtype=torch.float64).view(nz, 1, 1)
    fy = torch.fft.fftfreq(ny, d=1.0 / ny, device=dev, dtype=torch.float64).view(1, ny, 1)
    fx = torch.fft.fftfreq(nx, d=1.0 / nx, device=dev, dtype=torch.float64).view(1, 1, nx)
    shell = torch.floor(torch.sqrt(fz * fz + fy * fy + fx * fx) + 0.5).long().reshape(-1)
    vh = torch.fft.fftn(v, dim=(1, 2, 3)) / n
    e = 0.5 * (vh.real ** 2 + vh.imag ** 2).sum(0).reshape(-1)
    keep = shell < nshells
    return torch.zeros(nshells, dtype=e.dtype, device=dev).index_add(0, shell[keep], e[keep])


@dataclasses.dataclass
class RolloutConfig:
    nx: int
    ny: int
    nz: int
    nu: float
    eta: float
    d_i: float = 0.0
    b0: tuple = (0.0, 0.0, 0.0)
    storage: str = "f64"
    jmode: str = "moment"
    layout: str = "aa"
    nsteps: int = 10
    ckpt: int = 50
    force_u: Optional[torch.Tensor] = None
    force_b: Optional[torch.Tensor] = None
    recompute: str = "auto"    # "trace" | "state" | "auto" (trace where available)

    def uses_trace(self):
        available = self.jmode == "moment" and self.layout == "aa"
        if self.recompute == "trace" and not available:
            raise ValueError("trace recompute needs the moment route and the AA layout")
        return available and self.recompute != "state"


class FlameRollout(torch.autograd.Function):
    """(u0, b0, grad_u0, grad_b0, cfg) -> (u_T, B_T); grad_* may be None (no non-equilibrium
    initialisation, J = 0 in the initial Hall equilibrium)."""

    @staticmethod
    def forward(ctx, u0, b0, gu0, gb0, cfg: RolloutConfig):
        if (gu0 is None) != (gb0 is None):
            raise ValueError("pass both initial gradients or neither")
        # without gradients the run starts at equilibrium (no non-equilibrium parts, J = 0)
        s = Solver(cfg.nx, cfg.ny, cfg.nz, cfg.nu, cfg.eta, cfg.d_i, cfg.b0, cfg.storage, cfg.jmode, cfg.layout,
                   u0.detach(), b0.detach(), None if gu0 is None else gu0.detach(),
                   None if gb0 is None else gb0.detach(), cfg.force_u, cfg.force_b, init_noneq=gu0 is not None)
        trace = cfg.uses_trace()
        ckpts = []
        done = 0
        while done < cfg.nsteps:
            if trace:
                lat = torch.empty(L.flame_trace_bytes(s.ctx), dtype=torch.uint8, device=s.device)
                L.flame_trace_export(s.ctx, lat.data_ptr())
                ckpts.append((lat, done))
            else:
                f, g = s.get_populations(deviations=True)
                ckpts.append(((f.clone(), g.clone()), done))
            k = min(cfg.ckpt, cfg.nsteps - done)
            s.step(k)
            done += k
        _, u, B, _, _ = s.fields()
        ctx.solver, ctx.ckpts, ctx.cfg = s, ckpts, cfg
        ctx.has_grads = (gu0 is not None, gb0 is not None)
        ctx.save_for_backward(u0.detach(), b0.detach(), *(t.detach() for t in (gu0, gb0) if t is not None))
        return u.clone(), B.clone()

    @staticmethod
    def backward(ctx, g_u, g_B):
        s, cfg = ctx.solver, ctx.cfg
        saved = ctx.saved_tensors
        u0, b0 = saved[0], saved[1]
        rest = list(saved[2:])
        gu0 = rest.pop(0) if ctx.has_grads[0] else None
        gb0 = rest.pop(0) if ctx.has_grads[1] else None
        dev = s.device
        adt = torch.float64 if cfg.storage == "f64" else torch.float32
        n = s.n
        lam = torch.empty(48 * n, dtype=adt, device=dev)
        lam2 = torch.empty_like(lam)
        lam_j = torch.empty(3 * n, dtype=adt, device=dev) if cfg.jmode == "stencil" else None
        ptr = lambda t: 0 if t is None else t.data_ptr()  # noqa: E731
        # the forward left the solver at the final state
        gu = None if g_u is None else g_u.to(dev, torch.float64).contiguous()
        gB = None if g_B is None else g_B.to(dev, torch.float64).contiguous()
        L.flame_adjoint_fields(s.ctx, ptr(gu), ptr(gB), lam.data_ptr())
        seg = min(cfg.ckpt, cfg.nsteps)
        if cfg.uses_trace():
            pool = torch.empty((max(seg - 1, 0), L.flame_trace_bytes(s.ctx)), dtype=torch.uint8, device=dev)
            for lat0, start in reversed(ctx.ckpts):
                length = min(cfg.ckpt, cfg.nsteps - start)
                chain = [lat0] + [pool[k] for k in range(length - 1)]
                for k in range(length - 1):
                    L.flame_trace_step(s.ctx, chain[k].data_ptr(), chain[k + 1].data_ptr())
                for k in reversed(range(length)):
                    L.flame_adjoint_trace_step(s.ctx, chain[k].data_ptr(), lam.data_ptr(), lam2.data_ptr())
                    lam, lam2 = lam2, lam
        else:
            states = torch.empty((seg, 51 * n), dtype=adt, device=dev)
            for (f, g), start in reversed(ctx.ckpts):
                length = min(cfg.ckpt, cfg.nsteps - start)
                s.set_populations(f, g, deviations=True)
                for k in range(length):
                    L.flame_step_save(s.ctx, states[k].data_ptr())
                for k in reversed(range(length)):
                    L.flame_adjoint_step(s.ctx, states[k].data_ptr(), lam.data_ptr(), lam2.data_ptr(), ptr(lam_j))
                    lam, lam2 = lam2, lam
        out_u = torch.empty_like(u0)
        out_b = torch.empty_like(b0)
        out_gu = None if gu0 is None else torch.empty_like(gu0)
        out_gb = None if gb0 is None else torch.empty_like(gb0)
        L.flame_adjoint_init(s.ctx, lam.data_ptr(), u0.data_ptr(), b0.data_ptr(), ptr(gu0), ptr(gb0),
                             out_u.data_ptr(), out_b.data_ptr(), ptr(out_gu), ptr(out_gb))
        s.stream.synchronize()
        return out_u, out_b, out_gu, out_gb, None


def rollout(u0, b0, cfg: RolloutConfig, noneq: bool = True):
    """Final (u_T, B_T) of a run started from u0, b0 (3, nz, ny, nx) float64 tensors on the
    device; with ``noneq`` the initial non-equilibrium parts use spectral gradients of u0, b0,
    so gradients flow through them too."""
    gu0 = spectral_gradient(u0) if noneq else None
    gb0 = spectral_gradient(b0) if noneq else None
    return FlameRollout.apply(u0, b0, gu0, gb0, cfg)


def spectrum_misfit(B, target, nshells):
    """Squared misfit of the magnetic shell spectrum over shells 1..nshells-1."""
    e = shell_spectrum(B, nshells)
    return ((e[1:] - target[1:]) ** 2).sum()
