"""Pins of the oracle's lattice constants and equilibria against closed-form identities.

Lattice: paper Sec. 3.1-3.2 and App. A. Equilibria: App. A (sixth-order Hermite f^(0)),
Sec. 3.1 (Maxwell-stress upgrade and its stated second moment), Sec. 3.2 (Hall equilibrium
and its first moment).
"""

import itertools

import torch

from oracle import equilibrium as eq
from oracle.lattice import C, C2, CS2, W, WM, XI, opposite

torch.manual_seed(0)


def test_d3q27_weights_and_isotropy():
    assert torch.isclose(W.sum(), torch.tensor(1.0, dtype=W.dtype), atol=1e-15)
    # second and fourth moments of the weights: c_s^2 delta and c_s^4 (3 delta delta sym.)
    for a, b in itertools.product(range(3), repeat=2):
        m2 = (W * C[:, a] * C[:, b]).sum()
        assert abs(m2 - (CS2 if a == b else 0.0)) < 1e-15
    assert abs((W * C[:, 0] ** 2 * C[:, 1] ** 2).sum() - 1.0 / 9.0) < 1e-15
    assert abs((W * C[:, 0] ** 4).sum() - 1.0 / 3.0) < 1e-15
    # the App. A listing holds every velocity of {-1,0,1}^3 once, opposites in pairs
    assert len({tuple(r.tolist()) for r in C}) == 27
    for i in range(27):
        assert torch.equal(C[opposite(i)], -C[i])


def test_app_a_edge_weight_misprint():
    # With App. A's edge weight 8/27 in place of 1/54 the weights cannot sum to one.
    w = W.clone()
    w[(C * C).sum(1) == 2] = 8.0 / 27.0
    assert w.sum() > 4.3


def test_d3q7_constants():
    assert torch.isclose(WM.sum(), torch.tensor(1.0, dtype=WM.dtype))
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((WM * XI[:, a] * XI[:, b]).sum() - (C2 if a == b else 0.0)) < 1e-16
    # node coincidence 2C = sqrt(3) c_s
    assert abs(4 * C2 - 3 * CS2) < 1e-15


def _product_form(rho, U):
    """Textbook D1Q3 equilibrium per axis (moments rho, rho u, rho (u^2 + 1/3)), multiplied."""
    out = []
    for i in range(27):
        v = rho.clone()
        for a in range(3):
            u = U[a]
            c = int(C[i, a])
            v = v * ((2.0 / 3.0 - u * u) if c == 0 else 0.5 * (1.0 / 3.0 + u * u + c * u))
        out.append(v)
    return torch.stack(out)


def test_hermite6_equals_product_form():
    rho = 1.0 + 0.1 * torch.randn(200, dtype=torch.float64)
    U = 0.2 * torch.randn(3, 200, dtype=torch.float64)
    assert torch.allclose(eq.f_eq(rho, U), _product_form(rho, U), rtol=0, atol=2e-16)


def _central_moments(f, U, p):
    cb = C.unsqueeze(-1) - U.unsqueeze(0)          # (27, 3, n)
    return (f * cb[:, 0] ** p[0] * cb[:, 1] ** p[1] * cb[:, 2] ** p[2]).sum(0)


def test_equilibrium_central_moments_are_maxwellian():
    rho = 1.0 + 0.05 * torch.randn(50, dtype=torch.float64)
    U = 0.1 * torch.randn(3, 50, dtype=torch.float64)
    f0 = eq.f_eq(rho, U)
    expect = {0: 1.0, 1: 0.0, 2: CS2}
    for p in itertools.product(range(3), repeat=3):
        want = rho * expect[p[0]] * expect[p[1]] * expect[p[2]]
        assert torch.allclose(_central_moments(f0, U, p), want, atol=1e-15), p


def test_maxwell_term_moments():
    B = 0.3 * torch.randn(3, 40, dtype=torch.float64)
    m = eq.maxwell_term(B)
    assert m.sum(0).abs().max() < 1e-15
    assert torch.einsum("in,ia->an", m, C).abs().max() < 1e-15
    b2 = (B * B).sum(0)
    for a, b in itertools.product(range(3), repeat=2):
        want = (0.5 * b2 if a == b else 0.0) - B[a] * B[b]
        got = (m * (C[:, a] * C[:, b]).unsqueeze(-1)).sum(0)
        assert torch.allclose(got, want, atol=1e-15)


def test_printed_maxwell_term_breaks_mass():
    # The Lorentz term as printed, (w / 2 c_s^4)(|B|^2 |c|^2 - (c.B)^2), adds 3|B|^2 of mass
    B = torch.tensor([[0.1], [0.2], [-0.3]], dtype=torch.float64)
    c2 = (C * C).sum(1, keepdim=True)
    cb = C @ B
    printed = W.unsqueeze(-1) / (2 * CS2 ** 2) * ((B * B).sum(0) * c2 - cb ** 2)
    assert abs(printed.sum() - 3 * (B * B).sum()) < 1e-15


def test_hall_equilibrium_moments():
    U = 0.1 * torch.randn(3, 30, dtype=torch.float64)
    B = 0.2 * torch.randn(3, 30, dtype=torch.float64)
    J = 0.05 * torch.randn(3, 30, dtype=torch.float64)
    a = 1.7
    g = eq.g_eq_hall(U, B, J, a)
    assert torch.allclose(g.sum(0), B, atol=1e-16)
    lam = torch.einsum("ia,ibn->abn", XI, g)
    V = U - a * J
    for x, y in itertools.product(range(3), repeat=2):
        assert torch.allclose(lam[x, y], V[x] * B[y] - B[x] * V[y], atol=1e-16)
    assert (lam[0, 0] + lam[1, 1] + lam[2, 2]).abs().max() < 1e-16
