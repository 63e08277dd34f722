"""Trace lattices (moment route, AA layout), through the C ABI:
  * exporting the state and stepping the exported lattice with flame_trace_step reproduces the
    context's own steps bitwise (every storage, ragged forced grid) and leaves the context
    untouched;
  * the routes and layouts the trace entry points do not serve are refused with
    FLAME_E_UNSUPPORTED, bad arguments with FLAME_E_INVAL, and nothing is launched.

The stencil route and the two-lattice (AB) layout are switched off in the library: the first GPU
run of each (export from a two-copy magnetic set, the pull z-marching step) ended in a memory
fault whose cause has not been found; a CPU build of the same kernels under AddressSanitizer
shows no out-of-bounds access for either. Their cases stay below, skipped."""

import pytest
import torch

from parity_helpers import Case, gpu_solver

pytestmark = pytest.mark.gpu

CASES = {
    "moment": Case(13, 10, 9, jmode="moment", forced=True, seed=11),
    "stencil": Case(13, 10, 9, jmode="stencil", forced=True, seed=12),
}

OFF = pytest.mark.skip(reason="switched off: its first GPU run ended in a memory fault of unknown cause")


@pytest.mark.parametrize("layout", ["aa", pytest.param("ab", marks=OFF)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("jmode", ["moment", pytest.param("stencil", marks=OFF)])
def test_trace_reproduces_steps(jmode, storage, layout):
    from paper_2212_11024_amd import _lib as L
    print(f"[trace] {jmode} {storage} {layout}", flush=True)
    s = gpu_solver(CASES[jmode], storage, layout)
    s.step(3)                                  # odd: the AA sets sit in swapped slots
    nb = L.flame_trace_bytes(s.ctx)
    assert nb == 48 * s.n * {"f64": 8, "f32": 4, "f16": 2}[storage]
    k = 6
    lat = torch.empty((k + 1, nb), dtype=torch.uint8, device=s.device)
    L.flame_trace_export(s.ctx, lat[0].data_ptr())
    for t in range(k):
        L.flame_trace_step(s.ctx, lat[t].data_ptr(), lat[t + 1].data_ptr())
    assert s.steps == 3
    before = torch.empty(nb, dtype=torch.uint8, device=s.device)
    L.flame_trace_export(s.ctx, before.data_ptr())
    s.step(k)
    after = torch.empty(nb, dtype=torch.uint8, device=s.device)
    L.flame_trace_export(s.ctx, after.data_ptr())
    torch.cuda.synchronize()
    assert torch.equal(before, lat[0])         # the trace steps left the context alone
    assert torch.equal(after, lat[k])          # and reproduce its steps bitwise


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_trace_reproduces_steps_at_benchmark_size(storage):
    """The same at the benchmark's size and launch configuration (512^3 forced, moment J, AA):
    the exported lattice stepped twice with flame_trace_step (a pull step over arrays of stride
    n, in the node-local kernel with the addressing it takes for this storage) equals the
    context's own two steps bit for bit."""
    import bench
    from paper_2212_11024_amd import _lib as L
    print(f"[trace] 512^3 {storage}", flush=True)
    s = bench.make_solver(512, storage, "moment", "aa")
    s.step(1)
    nb = L.flame_trace_bytes(s.ctx)
    lat = torch.empty((3, nb), dtype=torch.uint8, device=s.device)
    L.flame_trace_export(s.ctx, lat[0].data_ptr())
    for t in range(2):
        L.flame_trace_step(s.ctx, lat[t].data_ptr(), lat[t + 1].data_ptr())
    s.step(2)
    L.flame_trace_export(s.ctx, lat[0].data_ptr())
    torch.cuda.synchronize()
    assert torch.equal(lat[0], lat[2])
    s.close()


def test_trace_argument_errors():
    """Host-side refusals only: no kernel is launched by any trace call below."""
    from paper_2212_11024_amd import _lib as L
    s = gpu_solver(Case(8, 6, 5, jmode="moment"), "f32", "aa")
    nb = L.flame_trace_bytes(s.ctx)
    lat = torch.empty((2, nb), dtype=torch.uint8, device=s.device)
    a, b = lat[0].data_ptr(), lat[1].data_ptr()
    with pytest.raises(L.FlameError):
        L.flame_trace_step(s.ctx, 0, b)                            # no source
    with pytest.raises(L.FlameError):
        L.flame_trace_step(s.ctx, a, a)                            # in place
    with pytest.raises(L.FlameError):
        L.flame_trace_step(s.ctx, a, 0)                            # no destination
    with pytest.raises(L.FlameError):
        L.flame_trace_export(s.ctx, 0)
    s.close()
    for jmode, layout in (("stencil", "aa"), ("moment", "ab")):
        s = gpu_solver(Case(8, 6, 5, jmode=jmode), "f32", layout)
        lat = torch.empty((2, L.flame_trace_bytes(s.ctx)), dtype=torch.uint8, device=s.device)
        with pytest.raises(L.FlameError) as e:
            L.flame_trace_export(s.ctx, lat[0].data_ptr())        # switched off
        assert e.value.code == L.FLAME_E_UNSUPPORTED
        for call in (lambda: L.flame_trace_step(s.ctx, lat[0].data_ptr(), lat[1].data_ptr()),
                     lambda: L.flame_adjoint_trace_step(s.ctx, lat[0].data_ptr(), lat[1].data_ptr(),
                                                        lat[0].data_ptr())):
            with pytest.raises(L.FlameError) as e:
                call()                                             # switched off, nothing launched
            assert e.value.code == L.FLAME_E_UNSUPPORTED
        s.close()
