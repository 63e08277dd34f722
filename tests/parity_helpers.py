"""Shared helpers for the GPU-vs-oracle parity tests: seeded inputs fed to both sides and
the deviation-norm comparison. Imports the oracle (test infrastructure) and the product
binding side by side; neither imports the other."""

from __future__ import annotations

import dataclasses

import numpy as np
import torch

import synthetic
from oracle import extended, scheme


@dataclasses.dataclass
class Case:
    nx: int
    ny: int
    nz: int
    nu: float = 0.02
    eta: float = 0.03
    d_i: float = 2.0
    b0: tuple = (0.01, -0.02, 0.05)
    jmode: str = "moment"
    rms: float = 0.02
    forced: bool = False
    seed: int = 0
    kmax: int = 2
    ic: str = "shell"      # "shell": seeded shell fields; "orszag_tang": u amplitude rms, B amplitude 0.8 rms
    collision: str = "central"   # fluid collision: "central" or "bgk"
    magnetic: str = "hall"       # magnetic equilibrium: "hall" or "emhd"
    fluid_lattice: str = "d3q27"
    magnetic_lattice: str = "d3q7"

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)


def inputs(case: Case, device="cpu"):
    """u, grad u, b, grad b, F, S (float64) on ``device``; F, S are None when unforced."""
    if case.ic == "orszag_tang":
        fu_ic, fb_ic = synthetic.orszag_tang(case.rms, 0.8 * case.rms)
    else:
        km = min(case.kmax, (min(case.shape) - 1) // 2)
        fu_ic = synthetic.shell_field(case.seed, 1, km, case.rms)
        fb_ic = synthetic.shell_field(case.seed + 1, 1, km, case.rms)
    u, gu = synthetic.evaluate(fu_ic, case.shape, device)
    b, gb = synthetic.evaluate(fb_ic, case.shape, device)
    fu = fb = None
    if case.forced:
        fu, _ = synthetic.evaluate(synthetic.shell_field(case.seed + 2, 0, 1, 1e-4, "radius"), case.shape, device,
                                   gradient=False)
        fb, _ = synthetic.evaluate(synthetic.shell_field(case.seed + 3, 0, 1, 1e-4, "radius"), case.shape, device,
                                   gradient=False)
    return u, gu, b, gb, fu, fb


def oracle_params(case: Case, fu=None, fb=None, route="closed"):
    return scheme.Params(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, case.jmode, route,
                         fu, fb, collision=case.collision, magnetic=case.magnetic,
                         fluid_lattice=case.fluid_lattice, magnetic_lattice=case.magnetic_lattice)


def oracle_run(case: Case, steps: int, route="closed", noneq=True, ftype=torch.float64):
    """Oracle state after ``steps`` from the seeded inputs (forcing cast through ftype so both
    sides see the same forcing values)."""
    u, gu, b, gb, fu, fb = inputs(case)
    if fu is not None:
        fu = fu.to(ftype).to(torch.float64)
        fb = fb.to(ftype).to(torch.float64)
    p = oracle_params(case, fu, fb, route)
    st = scheme.init_state(p, u, b, gu, gb, noneq=noneq)
    return p, scheme.step(st, p, steps)


def gpu_solver(case: Case, storage="f64", layout="aa", noneq=True):
    from paper_2212_11024_amd.solver import Solver
    u, gu, b, gb, fu, fb = inputs(case)
    return Solver(case.nx, case.ny, case.nz, case.nu, case.eta, case.d_i, case.b0, storage, case.jmode, layout,
                  u, b, gu, gb, fu, fb, init_noneq=noneq, collision=case.collision, magnetic=case.magnetic,
                  fluid_lattice=case.fluid_lattice, magnetic_lattice=case.magnetic_lattice)


def deviation_error(solver, p, st):
    """Relative L2 error of the GPU populations against the FP64 oracle state, both measured
    as deviations from the rest state f^mhd(0)(1, 0, b0), g = W b0, over all 48 arrays."""
    rest = scheme.rest_state(p)
    df, dg = solver.get_populations(deviations=True)
    of = st.f - rest.f
    og = st.g - rest.g
    num = ((df.cpu() - of) ** 2).sum() + ((dg.cpu() - og) ** 2).sum()
    den = (of ** 2).sum() + (og ** 2).sum()
    return float((num / den).sqrt())


def extended_run(case: Case, steps: int, ftype=torch.float64, noneq=True):
    """The same run in extended precision: (deviation f, deviation g) as longdouble arrays."""
    u, gu, b, gb, fu, fb = inputs(case)
    if fu is not None:
        fu = fu.to(ftype).to(torch.float64)
        fb = fb.to(ftype).to(torch.float64)
    xp = extended.Params(oracle_params(case, fu, fb))
    f, g = extended.init_state(xp, u, b, gu, gb, noneq=noneq)
    f, g = extended.step(f, g, xp, steps)
    fr, gr = extended.rest_state(xp, f.shape[1:])
    return f - fr, g - gr


def extended_error(solver, ref):
    """Relative L2 error of the GPU deviations against an extended-precision reference."""
    xf, xg = ref
    df, dg = solver.get_populations(deviations=True)
    df = df.cpu().numpy().astype(np.longdouble)
    dg = dg.cpu().numpy().astype(np.longdouble)
    num = ((df - xf) ** 2).sum() + ((dg - xg) ** 2).sum()
    den = (xf ** 2).sum() + (xg ** 2).sum()
    return float(np.sqrt(num / den))


def neighbourhood(centres, n):
    """Linear indices of the periodic 5^3 boxes around (x, y, z) centres on an n^3 grid."""
    off = np.arange(-2, 3)
    zz, yy, xx = np.meshgrid(off, off, off, indexing="ij")
    out = []
    for x, y, z in centres:
        out.append(((((z + zz) % n) * n + (y + yy) % n) * n + (x + xx) % n).reshape(-1))
    return np.concatenate(out)


def sampled_step_error(solver, centres, n, nu, eta, d_i, b0, jmode="moment", force=None, collision="central",
                       magnetic="hall", fluid_lattice="d3q27", magnetic_lattice="d3q7"):
    """One step of the GPU run checked on sampled nodes: the pre-step populations of each centre's
    periodic 5^3 neighbourhood are read back, the oracle steps that box once (the centre depends
    only on nodes within two cells), and the centre's post-step populations are compared. force:
    the (fu, fb) fields as the kernel sees them (float64 tensors (3, n, n, n)), or None.
    Returns (relative L2 error over the centres, worst single centre)."""
    nb_np = neighbourhood(centres, n)
    nb = torch.as_tensor(nb_np, device=solver.device)
    mid = torch.as_tensor([((z * n + y) * n + x) for x, y, z in centres], device=solver.device)
    k, q, m = len(centres), solver.q, solver.m
    kw = dict(collision=collision, magnetic=magnetic, fluid_lattice=fluid_lattice, magnetic_lattice=magnetic_lattice)
    rest = scheme.rest_state(scheme.Params(5, 5, 5, nu, eta, d_i, b0, jmode, "closed", **kw))
    pre = solver.gather(nb).cpu().view(k, 125, q + 3 * m)
    fpre = bpre = None
    if force is not None:
        fpre = force[0].flatten(1)[:, nb].cpu().view(3, k, 125)
        bpre = force[1].flatten(1)[:, nb].cpu().view(3, k, 125)
    solver.step(1)
    post = solver.gather(mid, deviations=True).cpu()
    num = den = worst = 0.0
    for i in range(k):
        f = pre[i, :, :q].T.reshape(q, 5, 5, 5).contiguous()
        g = pre[i, :, q:].T.reshape(m, 3, 5, 5, 5).contiguous()
        fu = None if fpre is None else fpre[:, i].reshape(3, 5, 5, 5)
        fb = None if bpre is None else bpre[:, i].reshape(3, 5, 5, 5)
        p = scheme.Params(5, 5, 5, nu, eta, d_i, b0, jmode, "closed", fu, fb, **kw)
        st = scheme.step(scheme.State(f, g), p, 1)
        want = torch.cat([(st.f - rest.f)[:, 2, 2, 2], (st.g - rest.g)[:, :, 2, 2, 2].reshape(-1)])
        d = float(((post[i] - want) ** 2).sum())
        w = float((want ** 2).sum())
        num += d
        den += w
        worst = max(worst, (d / w) ** 0.5)
    return (num / den) ** 0.5, worst
