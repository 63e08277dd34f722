"""The kernels' per-node arithmetic (compiled for the host from the same header the HIP
kernels use) against the oracle: forward collision, and the hand-written reverse pass against
torch autograd through the oracle's collision (the definition route, T-matrix)."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from oracle import collision, current, equilibrium, scheme
from oracle.lattice import C, WM, XI, omega_fluid, omega_magnetic

HERE = os.path.dirname(os.path.abspath(__file__))
D = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def hc(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("hc") / "hc.so")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-host-only", "-x", "hip",
                    os.path.join(HERE, "hostcheck", "flame_hostcheck.hip"), "-o", out], check=True,
                   stderr=subprocess.DEVNULL)
    lib = ctypes.CDLL(out)
    lib.hc_collide.argtypes = [ctypes.c_int] + [D] * 9
    lib.hc_collide_vjp.argtypes = [ctypes.c_int] + [D] * 11
    I = ctypes.POINTER(ctypes.c_int)
    lib.hc_init.argtypes = [D] * 7 + [I, D, D]
    lib.hc_init_vjp.argtypes = [D] * 6 + [I] + [D] * 6
    lib.hc_variant_collide.argtypes = [ctypes.c_int] * 4 + [D] * 7
    lib.hc_buffer_ok.argtypes = [ctypes.c_int] * 5
    lib.hc_row_threads.argtypes = [ctypes.c_int] * 2
    lib.hc_row_threads.restype = ctypes.c_uint
    return lib


def _p(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(D)


def _case(rng, forced=True):
    nu, eta, d_i = rng.uniform(0.005, 0.05), rng.uniform(0.005, 0.05), rng.uniform(0.0, 6.0)
    b0 = rng.normal(0, 0.05, 3)
    params = scheme.Params(1, 1, 1, nu, eta, d_i, tuple(b0))
    rest = scheme.rest_state(params)
    U = rng.normal(0, 0.04, 3)
    B = b0 + rng.normal(0, 0.05, 3)
    f = equilibrium.f_mhd_eq(torch.ones(1, dtype=torch.float64), torch.tensor(U).view(3, 1),
                             torch.tensor(B).view(3, 1))[:, 0].numpy() + rng.normal(0, 2e-4, 27)
    g = (WM.view(7, 1) * torch.tensor(B).view(1, 3)).numpy() + rng.normal(0, 3e-3, (7, 3))
    F = rng.normal(0, 1e-4, 3) if forced else np.zeros(3)
    S = rng.normal(0, 1e-4, 3) if forced else np.zeros(3)
    J = rng.normal(0, 0.01, 3)
    kp = np.array([omega_fluid(nu), omega_magnetic(eta), d_i, *b0])
    return params, rest, f, g, F, S, J, kp


def _oracle_node(f, g, F, S, params, J=None):
    """Oracle collision of one node (full values) as a differentiable torch function."""
    f2 = f.view(27, 1)
    g2 = g.view(7, 3, 1)
    rho = f2.sum(0)
    mom = torch.einsum("in,ia->an", f2, C) + 0.5 * F.view(3, 1)
    U = mom / rho
    B = g2.sum(0) + 0.5 * S.view(3, 1)
    lam = torch.einsum("ia,ibn->abn", XI, g2)
    if J is None:
        J = current.current_moment(lam, U, B, params.d_i, params.omega_b)
    else:
        J = J.view(3, 1)
    fs = collision.collide_T(f2, rho, U, B, params.omega, F=F.view(3, 1))
    gs = g2 - params.omega_b * (g2 - equilibrium.g_eq_hall(U, B, J, params.d_i))
    gs = gs + (1.0 - 0.5 * params.omega_b) * WM.view(7, 1, 1) * S.view(1, 3, 1)
    return fs.reshape(27), gs.reshape(21)


@pytest.mark.parametrize("grouped", [0, 1])
@pytest.mark.parametrize("moment", [1, 0])
def test_forward_collision_matches_oracle(hc, moment, grouped):
    rng = np.random.default_rng(10 + moment)
    for _ in range(20):
        params, rest, f, g, F, S, J, kp = _case(rng)
        fr, gr = rest.f[:, 0, 0, 0].numpy(), rest.g[:, :, 0, 0, 0].reshape(21).numpy()
        df, pdf = _p(f - fr)
        dg, pdg = _p(g.reshape(21) - gr)
        fo, pfo = _p(np.zeros(27))
        go, pgo = _p(np.zeros(21))
        jo, pjo = _p(np.zeros(3))
        hc.hc_collide(moment | (grouped << 1), pdf, pdg, _p(F)[1], _p(S)[1], _p(J)[1], _p(kp)[1], pfo, pgo, pjo)
        t = lambda a: torch.tensor(a, dtype=torch.float64)  # noqa: E731
        ofs, ogs = _oracle_node(t(f), t(g), t(F), t(S), params, None if moment else t(J))
        assert np.abs(fo - (ofs.numpy() - fr)).max() < 1e-15
        assert np.abs(go - (ogs.numpy() - gr)).max() < 1e-15


@pytest.mark.parametrize("moment", [1, 0])
def test_reverse_pass_matches_autograd(hc, moment):
    rng = np.random.default_rng(20 + moment)
    for _ in range(20):
        params, rest, f, g, F, S, J, kp = _case(rng)
        fr, gr = rest.f[:, 0, 0, 0].numpy(), rest.g[:, :, 0, 0, 0].reshape(21).numpy()
        mf = rng.normal(0, 1, 27)
        mg = rng.normal(0, 1, 21)
        tf = torch.tensor(f, dtype=torch.float64, requires_grad=True)
        tg = torch.tensor(g, dtype=torch.float64, requires_grad=True)
        tJ = torch.tensor(J, dtype=torch.float64, requires_grad=True)
        t = lambda a: torch.tensor(a, dtype=torch.float64)  # noqa: E731
        ofs, ogs = _oracle_node(tf, tg, t(F), t(S), params, None if moment else tJ)
        loss = (ofs * t(mf)).sum() + (ogs * t(mg)).sum()
        inputs = (tf, tg) if moment else (tf, tg, tJ)
        grads = torch.autograd.grad(loss, inputs)
        lf, plf = _p(np.zeros(27))
        lg, plg = _p(np.zeros(21))
        lJ, plJ = _p(np.zeros(3))
        hc.hc_collide_vjp(moment, _p(f - fr)[1], _p(g.reshape(21) - gr)[1], _p(F)[1], _p(S)[1], _p(J)[1],
                          _p(kp)[1], _p(mf)[1], _p(mg)[1], plf, plg, plJ)
        scale = float(max(grads[0].abs().max(), grads[1].abs().max()))
        assert np.abs(lf - grads[0].numpy()).max() < 1e-12 * scale
        assert np.abs(lg - grads[1].reshape(21).numpy()).max() < 1e-12 * scale
        if moment:
            assert np.abs(lJ).max() == 0.0
        else:
            assert np.abs(lJ - grads[2].numpy()).max() < 1e-12 * max(1.0, float(grads[2].abs().max()))


def _oracle_init(u, b, G, H, F, S, params, flags):
    """Oracle initial state of one node (full values) as a differentiable torch function."""
    p = scheme.Params(1, 1, 1, params.nu, params.eta, params.d_i, params.b0, "moment", "T",
                      F.view(3, 1, 1, 1), S.view(3, 1, 1, 1))
    st = scheme.init_state(p, u.view(3, 1, 1, 1), b.view(3, 1, 1, 1),
                           G.view(3, 3, 1, 1, 1) if flags[0] else None,
                           H.view(3, 3, 1, 1, 1) if flags[2] else None, noneq=bool(flags[0] or flags[1]))
    return st.f.reshape(27), st.g.reshape(21)


@pytest.mark.parametrize("flags", [(1, 1, 1), (0, 0, 1), (0, 0, 0)])
def test_initial_state_and_its_reverse_pass(hc, flags):
    rng = np.random.default_rng(30 + sum(flags))
    fl = (ctypes.c_int * 3)(*flags)
    for _ in range(10):
        params, rest, _, _, F, S, _, kp = _case(rng)
        u = rng.normal(0, 0.03, 3)
        b = rng.normal(0, 0.03, 3)
        G = rng.normal(0, 0.01, (3, 3))
        H = rng.normal(0, 0.01, (3, 3))
        fr, gr = rest.f[:, 0, 0, 0].numpy(), rest.g[:, :, 0, 0, 0].reshape(21).numpy()
        fo, pfo = _p(np.zeros(27))
        go, pgo = _p(np.zeros(21))
        hc.hc_init(_p(u)[1], _p(b)[1], _p(G)[1], _p(H)[1], _p(F)[1], _p(S)[1], _p(kp)[1], fl, pfo, pgo)
        tu, tb, tG, tH = (torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (u, b, G, H))
        t = lambda a: torch.tensor(a, dtype=torch.float64)  # noqa: E731
        of, og = _oracle_init(tu, tb, tG, tH, t(F), t(S), params, flags)
        assert np.abs(fo - (of.detach().numpy() - fr)).max() < 1e-15
        assert np.abs(go - (og.detach().numpy() - gr)).max() < 1e-15
        lf = rng.normal(0, 1, 27)
        lg = rng.normal(0, 1, 21)
        loss = (of * t(lf)).sum() + (og * t(lg)).sum()
        grads = torch.autograd.grad(loss, (tu, tb, tG, tH), allow_unused=True)
        outs = [_p(np.zeros(n)) for n in (3, 3, 9, 9)]
        hc.hc_init_vjp(_p(u)[1], _p(b)[1], _p(G)[1], _p(H)[1], _p(F)[1], _p(kp)[1], fl, _p(lf)[1], _p(lg)[1],
                       *[o[1] for o in outs])
        for (arr, _), ref in zip(outs, grads):
            ref = np.zeros(arr.size) if ref is None else ref.numpy().reshape(-1)
            assert np.abs(arr - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("fl,ml,coll,mag", [("d3q19", "d3q7", "bgk", "hall"), ("d3q27", "d3q15", "central", "hall"),
                                            ("d3q27", "d3q27", "bgk", "emhd"), ("d3q19", "d3q27", "bgk", "emhd"),
                                            ("d3q19", "d3q15", "bgk", "hall")])
def test_variant_collision_matches_oracle(hc, fl, ml, coll, mag):
    """The lattice variants' node update (moments, J from the magnetic moments, fluid and magnetic
    collisions, forcing), compiled for the host from the kernels' header, against the oracle's
    collision of the same node."""
    from oracle.lattice import FLUID_LATTICES, MAGNETIC_LATTICES
    rng = np.random.default_rng(hash((fl, ml, coll, mag)) % 2 ** 32)
    flat, mlat = FLUID_LATTICES[fl], MAGNETIC_LATTICES[ml]
    for trial in range(5):
        nu, eta, d_i = rng.uniform(0.005, 0.05), rng.uniform(0.005, 0.05), rng.uniform(0.0, 6.0)
        b0 = rng.normal(0, 0.05, 3)
        F = rng.normal(0, 1e-4, 3)
        S = rng.normal(0, 1e-4, 3)
        p = scheme.Params(1, 1, 1, nu, eta, d_i, tuple(b0), "moment", "closed",
                          torch.tensor(F).view(3, 1, 1, 1), torch.tensor(S).view(3, 1, 1, 1), collision=coll,
                          magnetic=mag, fluid_lattice=fl, magnetic_lattice=ml)
        rest = scheme.rest_state(p)
        U = torch.tensor(rng.normal(0, 0.04, 3)).view(3, 1)
        B = torch.tensor(b0 + rng.normal(0, 0.05, 3)).view(3, 1)
        f = equilibrium.f_mhd_eq_lattice(torch.ones(1, dtype=torch.float64), U, B, flat)[:, 0].numpy()
        f = f + rng.normal(0, 2e-4, flat.q)
        g = (mlat.w.view(-1, 1) * B.view(1, 3)).numpy() + rng.normal(0, 3e-3, (mlat.q, 3))
        st = scheme.State(torch.tensor(f).view(flat.q, 1, 1, 1), torch.tensor(g).view(mlat.q, 3, 1, 1, 1))
        want = scheme.collide(st, p)
        kp = np.array([omega_fluid(nu), omega_magnetic(eta), d_i, *b0])
        fo = np.zeros(flat.q)
        go = np.zeros(mlat.q * 3)
        args = [_p(f - rest.f.reshape(-1).numpy())[1], _p(g.reshape(-1) - rest.g.reshape(-1).numpy())[1],
                _p(F)[1], _p(S)[1], _p(kp)[1], fo.ctypes.data_as(D), go.ctypes.data_as(D)]
        assert hc.hc_variant_collide(flat.q, mlat.q, int(coll == "bgk"), int(mag == "emhd"), *args) == 0
        df = fo + rest.f.reshape(-1).numpy() - want.f.reshape(-1).numpy()
        dg = go + rest.g.reshape(-1).numpy() - want.g.reshape(-1).numpy()
        assert np.abs(df).max() < 1e-15 and np.abs(dg).max() < 1e-15, (trial, np.abs(df).max(), np.abs(dg).max())


def test_launch_policy(hc):
    """Host logic of the launches: buffer resources only where every array the step touches ends
    at least 16 bytes below 4 GiB (populations of 2^30 FP32 values, exactly 4 GiB, and of 2^29
    FP64 values take the global addresses; 2^30 FP16 values, 2 GiB, and 512^3 FP64 do not; the
    [n] arrays of the arithmetic type count only when the launch reads forcing or writes a saved
    state), and row blocks never beyond the kernels' launch bound of 256 threads, whatever
    FLAME_ROW_THREADS asks for."""
    F64, F32, F16 = 0, 1, 2
    for arith in (0, 1):
        assert hc.hc_buffer_ok(512, 512, 512, F32, arith) == 1
        assert hc.hc_buffer_ok(512, 512, 512, F64, arith) == 1
        assert hc.hc_buffer_ok(1024, 1024, 1024, F32, arith) == 0
        assert hc.hc_buffer_ok(1024, 1024, 512, F64, arith) == 0      # 2^29 FP64 values: 4 GiB per array
        assert hc.hc_buffer_ok(1024, 1024, 511, F64, arith) == 1
    # 2^30 FP16 populations fit (2 GiB); an FP32 forcing or saved-state array of 2^30 values does not
    assert hc.hc_buffer_ok(1024, 1024, 1024, F16, 0) == 1
    assert hc.hc_buffer_ok(1024, 1024, 1024, F16, 1) == 0
    assert hc.hc_buffer_ok(1024, 1024, 1023, F16, 1) == 1
    assert hc.hc_row_threads(512, 0) == 256
    assert hc.hc_row_threads(100, 0) == 128
    assert hc.hc_row_threads(512, 128) == 128
    assert hc.hc_row_threads(512, 512) == 256
    assert hc.hc_row_threads(512, 4096) == 256
    assert hc.hc_row_threads(40, 192) == 64
