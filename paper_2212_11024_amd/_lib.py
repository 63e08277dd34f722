"""ctypes binding of libflame.so: the C entry points of include/flame.h under the same names.

Argument marshalling only; every step of the computation runs in the HIP library. Loading
fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflame.so")

FLAME_OK = 0
FLAME_E_INVAL = -1
FLAME_E_NOMEM = -2
FLAME_E_HIP = -3
FLAME_E_NONFINITE = -4
FLAME_E_UNSUPPORTED = -5
FLAME_E_UNSTABLE = -6
FLAME_W_CFL = 1

FLAME_F64, FLAME_F32, FLAME_F16 = 0, 1, 2
FLAME_J_MOMENT, FLAME_J_STENCIL = 0, 1
FLAME_LAYOUT_AB, FLAME_LAYOUT_AA = 0, 1
FLAME_COLLISION_CENTRAL, FLAME_COLLISION_BGK = 0, 1
FLAME_MAGNETIC_HALL, FLAME_MAGNETIC_EMHD = 0, 1
FLAME_FLUID_D3Q27, FLAME_FLUID_D3Q19 = 0, 1
FLAME_MAGNETIC_D3Q7, FLAME_MAGNETIC_D3Q15, FLAME_MAGNETIC_D3Q27 = 0, 1, 2
FLAME_NRED = 16

FLUID_COUNT = {FLAME_FLUID_D3Q27: 27, FLAME_FLUID_D3Q19: 19}
MAGNETIC_COUNT = {FLAME_MAGNETIC_D3Q7: 7, FLAME_MAGNETIC_D3Q15: 15, FLAME_MAGNETIC_D3Q27: 27}


class flame_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nu", ctypes.c_double), ("eta", ctypes.c_double), ("d_i", ctypes.c_double),
        ("b0", ctypes.c_double * 3),
        ("storage", ctypes.c_int32), ("jmode", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("init_noneq", ctypes.c_int32),
        ("force_u", ctypes.c_void_p), ("force_b", ctypes.c_void_p),
        ("collision", ctypes.c_int32), ("magnetic", ctypes.c_int32),
        ("fluid_lattice", ctypes.c_int32), ("magnetic_lattice", ctypes.c_int32),
    ]


_P = ctypes.c_void_p
_SIGNATURES = {
    "flame_storage_bytes": (ctypes.c_size_t, [ctypes.POINTER(flame_params)]),
    "flame_rest_populations": (ctypes.c_int32, [ctypes.POINTER(flame_params), ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double)]),
    "flame_init": (ctypes.c_int32, [ctypes.POINTER(flame_params), _P, _P, _P, _P, _P, ctypes.c_size_t, _P,
                                    ctypes.POINTER(_P)]),
    "flame_step": (ctypes.c_int32, [_P, ctypes.c_int64]),
    "flame_moments": (ctypes.c_int32, [_P, _P, _P, _P, _P, _P]),
    "flame_reduce": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_double)]),
    "flame_reduce_noalloc": (ctypes.c_int32, [_P, _P]),
    "flame_spectrum": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "flame_dissipation_spectrum": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.c_double)]),
    "flame_energy_transfer": (ctypes.c_int32, [_P, ctypes.c_int32] + [ctypes.POINTER(ctypes.c_double)] * 4),
    "flame_get_populations": (ctypes.c_int32, [_P, _P, ctypes.c_int32]),
    "flame_set_populations": (ctypes.c_int32, [_P, _P, ctypes.c_int32]),
    "flame_gather": (ctypes.c_int32, [_P, _P, ctypes.c_int64, _P, ctypes.c_int32]),
    "flame_step_save": (ctypes.c_int32, [_P, _P]),
    "flame_trace_bytes": (ctypes.c_size_t, [_P]),
    "flame_trace_export": (ctypes.c_int32, [_P, _P]),
    "flame_trace_step": (ctypes.c_int32, [_P, _P, _P]),
    "flame_adjoint_trace_step": (ctypes.c_int32, [_P, _P, _P, _P]),
    "flame_adjoint_step": (ctypes.c_int32, [_P, _P, _P, _P, _P]),
    "flame_adjoint_fields": (ctypes.c_int32, [_P, _P, _P, _P]),
    "flame_adjoint_init": (ctypes.c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "flame_step_count": (ctypes.c_int64, [_P]),
    "flame_cfl_number": (ctypes.c_double, [_P]),
    "flame_last_error": (ctypes.c_char_p, [_P]),
    "flame_destroy": (None, [_P]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libflame.so (once). Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2212_11024_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FlameError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"flame status {code}: {msg}")
        self.code = code


def _check(code: int, ctx=None) -> int:
    if code < 0:
        msg = load().flame_last_error(ctx)
        raise FlameError(code, msg.decode() if msg else "")
    return code


# ---------------------------------------------------------------- entry points (same names)

def flame_storage_bytes(params: flame_params) -> int:
    return int(load().flame_storage_bytes(ctypes.byref(params)))


def flame_rest_populations(params: flame_params):
    """(f_rest[q], g_rest[3 m]) as lists of floats (q = 27, m = 7 on the paper's velocity sets)."""
    q = FLUID_COUNT[params.fluid_lattice]
    m = MAGNETIC_COUNT[params.magnetic_lattice]
    f = (ctypes.c_double * q)()
    g = (ctypes.c_double * (3 * m))()
    _check(load().flame_rest_populations(ctypes.byref(params), f, g))
    return list(f), list(g)


def flame_init(params: flame_params, u: int, b: int, grad_u: int, grad_b: int, storage: int,
               storage_bytes: int, stream: int) -> tuple[int, int]:
    """Returns (status, ctx); raises FlameError on a negative status."""
    out = _P()
    code = load().flame_init(ctypes.byref(params), u, b, grad_u, grad_b, storage, storage_bytes, stream,
                             ctypes.byref(out))
    _check(code, None)
    return code, out.value


def flame_step(ctx: int, nsteps: int) -> int:
    return _check(load().flame_step(ctx, nsteps), ctx)


def flame_moments(ctx: int, rho: int, u: int, b: int, j: int, divb: int) -> int:
    return _check(load().flame_moments(ctx, rho, u, b, j, divb), ctx)


def flame_reduce(ctx: int, allow_nonfinite: bool = False):
    """(status, out[FLAME_NRED]). allow_nonfinite: a blown-up state (FLAME_E_NONFINITE or
    FLAME_E_UNSTABLE) is returned with its status instead of raising."""
    out = (ctypes.c_double * FLAME_NRED)()
    code = load().flame_reduce(ctx, out)
    if not (allow_nonfinite and code in (FLAME_E_NONFINITE, FLAME_E_UNSTABLE)):
        _check(code, ctx)
    return code, list(out)


def flame_reduce_noalloc(ctx: int, out: int) -> int:
    """Reductions into the device buffer out (double [FLAME_NRED]); asynchronous, allocates nothing."""
    return _check(load().flame_reduce_noalloc(ctx, out), ctx)


def flame_spectrum(ctx: int, field: int, nshells: int):
    out = (ctypes.c_double * nshells)()
    _check(load().flame_spectrum(ctx, field, nshells, out), ctx)
    return list(out)


def flame_dissipation_spectrum(ctx: int, field: int, nshells: int):
    out = (ctypes.c_double * nshells)()
    _check(load().flame_dissipation_spectrum(ctx, field, nshells, out), ctx)
    return list(out)


def flame_energy_transfer(ctx: int, nshells: int, hall: bool = False):
    out = [(ctypes.c_double * nshells)() for _ in range(4 if hall else 3)]
    _check(load().flame_energy_transfer(ctx, nshells, *out, *([] if hall else [None])), ctx)
    return [list(o) for o in out]


def flame_get_populations(ctx: int, dst: int, deviations: int = 0) -> int:
    return _check(load().flame_get_populations(ctx, dst, deviations), ctx)


def flame_set_populations(ctx: int, src: int, deviations: int = 0) -> int:
    return _check(load().flame_set_populations(ctx, src, deviations), ctx)


def flame_gather(ctx: int, cells: int, n: int, out: int, deviations: int = 0) -> int:
    return _check(load().flame_gather(ctx, cells, n, out, deviations), ctx)


def flame_step_save(ctx: int, state: int) -> int:
    return _check(load().flame_step_save(ctx, state), ctx)


def flame_trace_bytes(ctx: int) -> int:
    return int(load().flame_trace_bytes(ctx))


def flame_trace_export(ctx: int, lat: int) -> int:
    return _check(load().flame_trace_export(ctx, lat), ctx)


def flame_trace_step(ctx: int, src: int, dst: int) -> int:
    return _check(load().flame_trace_step(ctx, src, dst), ctx)


def flame_adjoint_trace_step(ctx: int, src: int, lam_next: int, lam: int) -> int:
    return _check(load().flame_adjoint_trace_step(ctx, src, lam_next, lam), ctx)


def flame_adjoint_step(ctx: int, state: int, lam_next: int, lam: int, lam_j: int) -> int:
    return _check(load().flame_adjoint_step(ctx, state, lam_next, lam, lam_j), ctx)


def flame_adjoint_fields(ctx: int, dl_du: int, dl_db: int, lam: int) -> int:
    return _check(load().flame_adjoint_fields(ctx, dl_du, dl_db, lam), ctx)


def flame_adjoint_init(ctx: int, lam0: int, u: int, b: int, grad_u: int, grad_b: int, g_u: int, g_b: int,
                       g_grad_u: int, g_grad_b: int) -> int:
    return _check(load().flame_adjoint_init(ctx, lam0, u, b, grad_u, grad_b, g_u, g_b, g_grad_u, g_grad_b), ctx)


def flame_step_count(ctx: int) -> int:
    return int(load().flame_step_count(ctx))


def flame_cfl_number(ctx: int) -> float:
    return float(load().flame_cfl_number(ctx))


def flame_last_error(ctx) -> str:
    msg = load().flame_last_error(ctx)
    return msg.decode() if msg else ""


def flame_destroy(ctx: int) -> None:
    load().flame_destroy(ctx)
