"""The allocation-free reductions, flame_reduce_noalloc, against flame_reduce through the C ABI:
both run the same kernels in the same fixed order, so the device results must equal the host
ones bit for bit. Two calls in a row on different contexts, the second on a smaller grid, so that
the second call runs over the partials the first one left in the shared static scratch; the first
grid is large enough to use every row of that scratch."""

import pytest
import torch

from parity_helpers import Case, gpu_solver

pytestmark = pytest.mark.gpu


def _noalloc(s):
    from paper_2212_11024_amd import _lib as L
    out = torch.full((L.FLAME_NRED,), float("nan"), dtype=torch.float64, device=s.device)
    L.flame_reduce_noalloc(s.ctx, out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu()


def test_noalloc_reduce_equals_reduce():
    from paper_2212_11024_amd import _lib as L
    cases = [(Case(96, 90, 64, jmode="moment", forced=True, seed=41), "f32"),
             (Case(9, 8, 7, jmode="stencil", seed=43), "f64")]
    for case, storage in cases:
        print(f"[noalloc] {case.shape} {storage}", flush=True)
        s = gpu_solver(case, storage, "aa")
        s.step(4)
        got = _noalloc(s)
        code, ref = L.flame_reduce(s.ctx)
        assert code == L.FLAME_OK
        ref = torch.tensor(ref, dtype=torch.float64)
        assert torch.equal(got.view(torch.int64), ref.view(torch.int64)), (got, ref)
        assert float(got[9]) > 0.5 * s.n       # total mass: the kernels really ran on this state
        s.close()


def test_noalloc_reduce_counts_nonfinite_nodes():
    from paper_2212_11024_amd import _lib as L
    s = gpu_solver(Case(13, 10, 9, jmode="moment", seed=45), "f32", "aa")
    f, g = s.get_populations()
    f = f.clone()
    f[5, 3, 2, 7] = float("nan")
    s.set_populations(f, g)
    got = _noalloc(s)
    code, ref = L.flame_reduce(s.ctx, allow_nonfinite=True)
    assert code == L.FLAME_E_NONFINITE and float(got[8]) == 1.0
    # bit patterns, so that the NaN slots compare too
    ref = torch.tensor(ref, dtype=torch.float64)
    assert torch.equal(got.view(torch.int64), ref.view(torch.int64)), (got, ref)
    s.close()
