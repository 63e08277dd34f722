"""Linear stability of the two J routes (FP64 oracle, CPU).

Small random perturbations of a uniform magnetised flow, at the dissipation of the 512^3
forced-turbulence workload (nu = eta = 0.001). With J from the central-difference curl of B the
Hall electric field enters the magnetic equilibrium explicitly, a forward step of a dispersive
(whistler) term, and the perturbations grow even far inside the whistler CFL bound; with J from
the first magnetic moment (the 3x3 solve of Sec. 3.2, which treats the J x B coupling
implicitly) they stay bounded, as they do for both routes without the Hall term. This pins the
measured fact that the stencil route cannot run the Hall workload for long at this dissipation."""

import math

import torch

from oracle import scheme

U0 = (0.02, 0.01, -0.015)
B0 = (0.03, -0.02, 0.04)          # |B| = 0.054


def _amplification(jmode, d_i, n=8, steps=(20, 80), nu=0.001):
    g = torch.Generator().manual_seed(1)
    p = scheme.Params(n, n, n, nu, nu, d_i, B0, jmode, "closed")
    u = torch.tensor(U0, dtype=torch.float64).view(3, 1, 1, 1) + 1e-8 * torch.randn(
        (3, n, n, n), dtype=torch.float64, generator=g)
    b = 1e-8 * torch.randn((3, n, n, n), dtype=torch.float64, generator=g)
    st = scheme.init_state(p, u, b, noneq=False)

    def size(st):
        _, U, B, _, _ = scheme.fields(st, p)
        return float((U - U.mean(dim=(1, 2, 3), keepdim=True)).norm() + (B - B.mean(dim=(1, 2, 3), keepdim=True)).norm())

    st = scheme.step(st, p, steps[0])
    a = size(st)
    st = scheme.step(st, p, steps[1] - steps[0])
    return size(st) / a


def test_stencil_route_hall_term_is_unstable_at_low_dissipation():
    cfl = math.pi * 2.0 * math.sqrt(sum(c * c for c in B0))
    assert cfl < 0.4                             # well inside the whistler CFL bound
    assert _amplification("stencil", 2.0) > 100.0


def test_moment_route_and_no_hall_stay_bounded():
    assert _amplification("moment", 2.0) < 2.0
    assert _amplification("stencil", 0.0) < 2.0
    assert _amplification("moment", 0.0) < 2.0
