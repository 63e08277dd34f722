// Adjoint of the time step (reverse mode): lam_t = (d step / d x_t)^T lam_{t+1}.
//
// A step is x_{t+1} = Stream(Collide(x_t)) with x the canonical (post-streaming) populations.
// Streaming moves population q from node y to y + c_q, so its transpose gathers: the adjoint of
// the post-collision population q at node y is lam_{t+1}[q] at y + c_q. The collision is
// node-local except, on the stencil route, through J = curl b, which couples a node to the field
// of its six face neighbours; that coupling is transposed in a second pass (the central-difference
// curl is its own transpose). Forward values are taken either from the state saved by the
// forward step (flame_step_save: the adjoint reads 51 values, gathers 48 and writes 48 per node)
// or, on the moment route, from a trace lattice (flame_adjoint_trace_step: the pre-collision
// state is pulled from the previous time level exactly as the forward step pulls it, and J is
// recomputed from it, so the recompute is one ordinary step and writes nothing extra).

#include "flame_access.h"
#include "flame_internal.h"

namespace flame {

template <typename R>
struct AdjArgs {
  const R* state;      // [48 + 3][n]: pre-collision deviations and J of the forward step
  const R* lam_next;   // [48][n]
  R* lam;              // [48][n]
  R* lam_j;            // [3][n] (stencil route)
  const R* force_u;
  const R* force_b;
  int nx, ny, nz;
  size_t n;
  PhysConst<R> k;
};

constexpr int kAdjThreads = 256;
// Minimum waves per SIMD the reverse-pass kernels are compiled for (0: the compiler's choice).
#ifndef FLAME_ADJ_WAVES_PER_EU
#define FLAME_ADJ_WAVES_PER_EU 0
#endif
#if FLAME_ADJ_WAVES_PER_EU > 0
#define FLAME_ADJ_BOUNDS __launch_bounds__(kAdjThreads, FLAME_ADJ_WAVES_PER_EU)
#else
#define FLAME_ADJ_BOUNDS __launch_bounds__(kAdjThreads)
#endif

// Keeps the scheduler from moving the gathers of the next step's adjoints above the forward
// recomputation, so the pre-collision populations are dead before those values arrive (fewer
// registers live at once). Off unless FLAME_ADJ_FENCE is set.
#ifndef FLAME_ADJ_FENCE
#define FLAME_ADJ_FENCE 0
#endif
__device__ __forceinline__ void adj_phase_fence() {
  if (FLAME_ADJ_FENCE) __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ size_t anode(int x, int y, int z, int nx, int ny) {
  return (static_cast<size_t>(z) * ny + y) * nx + x;
}

// Addressing: 32-bit node offsets (Rows, Planes) from the uniform array bases, by 64-bit global
// addresses. Buffer resources, which the forward step uses, raise these kernels' register count
// to the 256 limit (one wave per SIMD) and slow the moment-route adjoint by 40%; the 32-bit
// offsets alone took it from 0.257 to 0.245 ms per step at 128^3 FP32. The entry points refuse
// arrays of more than 4 GiB.
//
// The adjoints of the next time level, gathered along the streaming: population q of node x went
// to x + c_q, so its adjoint is lam_next[q] there.
template <Addr A, typename R>
__device__ __forceinline__ void gather_next(const R* lam_next, size_t n, const Rows& rw, const Planes& pl,
                                            R (&mf)[kQ], R (&mg)[kM]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i)
    mf[i] = ld<A>(lam_next + static_cast<size_t>(i) * n, rw.at(cq(i, 0), cq(i, 1)) + pl.at(cq(i, 2)));
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const uint32_t dn = rw.at(xim(i, 0), xim(i, 1)) + pl.at(xim(i, 2));
#pragma unroll
    for (int c = 0; c < 3; ++c) mg[i * 3 + c] = ld<A>(lam_next + static_cast<size_t>(kQ + i * 3 + c) * n, dn);
  }
}

template <typename R, bool MOMENT>
__global__ FLAME_ADJ_BOUNDS void adjoint_step_kernel(AdjArgs<R> a) {
  constexpr Addr A = Addr::Global;
  unsigned bx, by, bz;
  logical_block((a.nx + blockDim.x - 1) / blockDim.x, a.ny, a.nz, bx, by, bz);
  const int x = bx * blockDim.x + threadIdx.x, y = by, z = bz;
  if (x >= a.nx) return;
  const size_t n = a.n;
  const Rows rw(x, y, a.nx, a.ny);
  const Planes pl(z, a.nz, static_cast<uint32_t>(a.nx) * a.ny);
  const uint32_t cell = rw.at(0, 0) + pl.at(0);
  R F[3];
  VjpState<R> fw;
  {
    R f[kQ], g[kM], J[3], S[3];
#pragma unroll
    for (int q = 0; q < kQ; ++q) f[q] = ld<A>(a.state + static_cast<size_t>(q) * n, cell);
#pragma unroll
    for (int q = 0; q < kM; ++q) g[q] = ld<A>(a.state + static_cast<size_t>(kQ + q) * n, cell);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      J[c] = ld<A>(a.state + static_cast<size_t>(kQ + kM + c) * n, cell);
      F[c] = a.force_u ? ld<A>(a.force_u + static_cast<size_t>(c) * n, cell) : R(0);
      S[c] = a.force_b ? ld<A>(a.force_b + static_cast<size_t>(c) * n, cell) : R(0);
    }
    fw = vjp_forward<R, MOMENT>(f, g, F, S, J, a.k);
  }
  adj_phase_fence();
  R mf[kQ], mg[kM];
  gather_next<A>(a.lam_next, n, rw, pl, mf, mg);
  R lf[kQ], lg[kM], lJ[3];
  vjp_reverse<R, MOMENT>(fw, F, a.k, mf, mg, lf, lg, lJ);
#pragma unroll
  for (int q = 0; q < kQ; ++q) st<A>(a.lam + static_cast<size_t>(q) * n, cell, lf[q]);
#pragma unroll
  for (int q = 0; q < kM; ++q) st<A>(a.lam + static_cast<size_t>(kQ + q) * n, cell, lg[q]);
  if (!MOMENT) {
#pragma unroll
    for (int c = 0; c < 3; ++c) st<A>(a.lam_j + static_cast<size_t>(c) * n, cell, lJ[c]);
  }
}

// Moment route from a trace lattice: the step's pre-collision state is the lattice pulled.
template <typename S>
struct AdjTraceArgs {
  using R = typename Enc<S>::R;
  const S* src;        // trace lattice [48][n] (storage encoding)
  const R* lam_next;   // [48][n]
  R* lam;              // [48][n]
  const R* force_u;
  const R* force_b;
  int nx, ny, nz;
  size_t n;
  PhysConst<R> k;
};

template <typename S>
__global__ FLAME_ADJ_BOUNDS void adjoint_trace_kernel(AdjTraceArgs<S> a) {
  constexpr Addr A = Addr::Global;
  using E = Enc<S>;
  using R = typename E::R;
  unsigned bx, by, bz;
  logical_block((a.nx + blockDim.x - 1) / blockDim.x, a.ny, a.nz, bx, by, bz);
  const int x = bx * blockDim.x + threadIdx.x, y = by, z = bz;
  if (x >= a.nx) return;
  const size_t n = a.n;
  const Rows rw(x, y, a.nx, a.ny);
  const Planes pl(z, a.nz, static_cast<uint32_t>(a.nx) * a.ny);
  const uint32_t cell = rw.at(0, 0) + pl.at(0);
  R F[3];
  VjpState<R> fw;
  {
    // the step's pre-collision state pulled from the lattice, and the forward step's J recomputed
    // from it (moment route, same order of operations)
    R f[kQ], g[kM], Sb[3];
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      f[i] = E::dec(ld<A>(a.src + static_cast<size_t>(i) * n, rw.at(-cq(i, 0), -cq(i, 1)) + pl.at(-cq(i, 2))),
                    R(1.0 / E::fscale(i)));
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const uint32_t sn = rw.at(-xim(i, 0), -xim(i, 1)) + pl.at(-xim(i, 2));
#pragma unroll
      for (int c = 0; c < 3; ++c)
        g[i * 3 + c] = E::dec(ld<A>(a.src + static_cast<size_t>(kQ + i * 3 + c) * n, sn), R(1.0 / E::mscale(i)));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      F[c] = a.force_u ? ld<A>(a.force_u + static_cast<size_t>(c) * n, cell) : R(0);
      Sb[c] = a.force_b ? ld<A>(a.force_b + static_cast<size_t>(c) * n, cell) : R(0);
    }
    const R unused[3] = {R(0), R(0), R(0)};
    fw = vjp_forward<R, true>(f, g, F, Sb, unused, a.k);
  }
  adj_phase_fence();
  R mf[kQ], mg[kM];
  gather_next<A>(a.lam_next, n, rw, pl, mf, mg);
  R lf[kQ], lg[kM], lJ[3];
  vjp_reverse<R, true>(fw, F, a.k, mf, mg, lf, lg, lJ);
#pragma unroll
  for (int q = 0; q < kQ; ++q) st<A>(a.lam + static_cast<size_t>(q) * n, cell, lf[q]);
#pragma unroll
  for (int q = 0; q < kM; ++q) st<A>(a.lam + static_cast<size_t>(kQ + q) * n, cell, lg[q]);
}

// Stencil route: b_c of every magnetic population set feeds J of the six face neighbours; add
// curl(lam_J) (the transpose of the central-difference curl) to the adjoint of all 7 g_{i,c}.
template <typename R>
__global__ __launch_bounds__(kAdjThreads) void adjoint_curl_kernel(R* lam, const R* lam_j, int nx, int ny, int nz,
                                                                    size_t n) {
  unsigned bx, by, bz;
  logical_block((nx + blockDim.x - 1) / blockDim.x, ny, nz, bx, by, bz);
  const int x = bx * blockDim.x + threadIdx.x, y = by, z = bz;
  if (x >= nx) return;
  const size_t cell = anode(x, y, z, nx, ny);
  auto L = [&](int c, int dx, int dy, int dz) {
    return lam_j[static_cast<size_t>(c) * n + anode(wrap(x + dx, nx), wrap(y + dy, ny), wrap(z + dz, nz), nx, ny)];
  };
  const R cx = R(0.5) * (L(2, 0, 1, 0) - L(2, 0, -1, 0)) - R(0.5) * (L(1, 0, 0, 1) - L(1, 0, 0, -1));
  const R cy = R(0.5) * (L(0, 0, 0, 1) - L(0, 0, 0, -1)) - R(0.5) * (L(2, 1, 0, 0) - L(2, -1, 0, 0));
  const R cz = R(0.5) * (L(1, 1, 0, 0) - L(1, -1, 0, 0)) - R(0.5) * (L(0, 0, 1, 0) - L(0, 0, -1, 0));
  const R cc[3] = {cx, cy, cz};
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) lam[static_cast<size_t>(kQ + i * 3 + c) * n + cell] += cc[c];
}

// Adjoint of the initial state: d loss / d(u, b, grad u, grad b) from lam_0.
template <typename R>
struct InitAdjArgs {
  const R* lam0;
  const double* u;
  const double* b;
  const double* gu;
  const double* gb;
  const R* force_u;
  double* out_u;
  double* out_b;
  double* out_gu;
  double* out_gb;
  size_t n;
  PhysConst<double> k;
  InitFlags fl;
};

template <typename R>
__global__ __launch_bounds__(256) void init_vjp_kernel(InitAdjArgs<R> a) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.n) return;
  const size_t n = a.n;
  double u[3], b[3], G[3][3] = {}, H[3][3] = {}, F[3], lf[kQ], lg[kM];
  for (int c = 0; c < 3; ++c) {
    u[c] = a.u[c * n + cell];
    b[c] = a.b[c * n + cell];
    F[c] = a.force_u ? static_cast<double>(a.force_u[c * n + cell]) : 0.0;
  }
  if (a.gu)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) G[p][q] = a.gu[(p * 3 + q) * n + cell];
  if (a.gb)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) H[p][q] = a.gb[(p * 3 + q) * n + cell];
  for (int q = 0; q < kQ; ++q) lf[q] = static_cast<double>(a.lam0[q * n + cell]);
  for (int q = 0; q < kM; ++q) lg[q] = static_cast<double>(a.lam0[(kQ + q) * n + cell]);
  double ou[3], ob[3], oG[3][3], oH[3][3];
  init_node_vjp(u, b, G, H, F, a.k, a.fl, lf, lg, ou, ob, oG, oH);
  for (int c = 0; c < 3; ++c) {
    a.out_u[c * n + cell] = ou[c];
    a.out_b[c * n + cell] = ob[c];
  }
  if (a.out_gu)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) a.out_gu[(p * 3 + q) * n + cell] = oG[p][q];
  if (a.out_gb)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) a.out_gb[(p * 3 + q) * n + cell] = oH[p][q];
}

template <typename R>
static hipError_t adjoint_typed(const flame_ctx* c, const void* state, const void* lam_next, void* lam, void* lam_j) {
  AdjArgs<R> a;
  a.state = static_cast<const R*>(state);
  a.lam_next = static_cast<const R*>(lam_next);
  a.lam = static_cast<R*>(lam);
  a.lam_j = static_cast<R*>(lam_j);
  a.force_u = static_cast<const R*>(c->p.force_u);
  a.force_b = static_cast<const R*>(c->p.force_b);
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.nz = c->p.nz;
  a.n = c->n;
  a.k.omega = R(c->omega);
  a.k.omega_b = R(c->omega_b);
  a.k.alpha = R(c->p.d_i);
  for (int i = 0; i < 3; ++i) a.k.b0[i] = R(c->p.b0[i]);
  const unsigned tx = row_threads(c->p.nx);
  const dim3 grid(((c->p.nx + tx - 1) / tx) * c->p.ny * c->p.nz);
  if (c->p.jmode == FLAME_J_STENCIL) {
    hipLaunchKernelGGL((adjoint_step_kernel<R, false>), grid, dim3(tx), 0, c->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adjoint_curl_kernel<R>, grid, dim3(tx), 0, c->stream, a.lam, a.lam_j, a.nx, a.ny,
                       a.nz, a.n);
  } else {
    hipLaunchKernelGGL((adjoint_step_kernel<R, true>), grid, dim3(tx), 0, c->stream, a);
  }
  return hipGetLastError();
}

template <typename S>
static hipError_t adjoint_trace_typed(const flame_ctx* c, const void* src, const void* lam_next, void* lam) {
  using R = typename Enc<S>::R;
  AdjTraceArgs<S> a;
  a.src = static_cast<const S*>(src);
  a.lam_next = static_cast<const R*>(lam_next);
  a.lam = static_cast<R*>(lam);
  a.force_u = static_cast<const R*>(c->p.force_u);
  a.force_b = static_cast<const R*>(c->p.force_b);
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.nz = c->p.nz;
  a.n = c->n;
  a.k.omega = R(c->omega);
  a.k.omega_b = R(c->omega_b);
  a.k.alpha = R(c->p.d_i);
  for (int i = 0; i < 3; ++i) a.k.b0[i] = R(c->p.b0[i]);
  const unsigned tx = row_threads(a.nx);
  const dim3 grid(((a.nx + tx - 1) / tx) * a.ny * a.nz);
  hipLaunchKernelGGL(adjoint_trace_kernel<S>, grid, dim3(tx), 0, c->stream, a);
  return hipGetLastError();
}

template <typename R>
static hipError_t init_vjp_typed(const flame_ctx* c, const void* lam0, const double* u, const double* b,
                                 const double* gu, const double* gb, double* ou, double* ob, double* ogu,
                                 double* ogb) {
  InitAdjArgs<R> a;
  a.lam0 = static_cast<const R*>(lam0);
  a.u = u;
  a.b = b;
  a.gu = gu;
  a.gb = gb;
  a.force_u = static_cast<const R*>(c->p.force_u);
  a.out_u = ou;
  a.out_b = ob;
  a.out_gu = ogu;
  a.out_gb = ogb;
  a.n = c->n;
  a.k.omega = c->omega;
  a.k.omega_b = c->omega_b;
  a.k.alpha = c->p.d_i;
  for (int i = 0; i < 3; ++i) a.k.b0[i] = c->p.b0[i];
  a.fl.fluid_noneq = c->p.init_noneq && gu;
  a.fl.mag_noneq = c->p.init_noneq && gb;
  a.fl.has_H = gb != nullptr;
  hipLaunchKernelGGL(init_vjp_kernel<R>, dim3((c->n + 255) / 256), dim3(256), 0, c->stream, a);
  return hipGetLastError();
}

// Every [n] array of the arithmetic type within 4 GiB (32-bit byte offsets in the kernels).
static bool adjoint_arrays_fit(flame_ctx* c) {
  const size_t bytes = c->n * (c->p.storage == FLAME_F64 ? 8 : 4);
  if (bytes <= (size_t(1) << 32)) return true;
  c->err = "reverse mode: each [n] array of the arithmetic type must fit in 4 GiB";
  return false;
}

}  // namespace flame

using namespace flame;

extern "C" {

flame_status flame_step_save(flame_ctx* c, void* state) {
  if (!c) return FLAME_E_INVAL;
  if (!reverse_mode_built(c->p)) {
    c->err = "reverse mode is built for the paper's model only (central-moment fluid, Hall equilibrium, "
             "D3Q27 / D3Q7 velocity sets)";
    return FLAME_E_UNSUPPORTED;
  }
  if (!state) {
    c->err = "state is NULL";
    return FLAME_E_INVAL;
  }
  if (!adjoint_arrays_fit(c)) return FLAME_E_INVAL;
  const SetPtrs ptr = set_ptrs(c);
  hipError_t e = launch_step(c, ptr, c->stride, state);
  if (e != hipSuccess) {
    c->err = std::string("step kernel: ") + hipGetErrorString(e);
    return FLAME_E_HIP;
  }
  const bool two_f = c->p.layout == FLAME_LAYOUT_AB;
  const bool two_g = mag_two_lattice(c->p);
  if (two_f || two_g) c->cur ^= 1;
  if (!two_f || !two_g) c->parity ^= 1;
  c->steps += 1;
  return FLAME_OK;
}

flame_status flame_trace_step(flame_ctx* c, const void* src, void* dst) {
  if (!c) return FLAME_E_INVAL;
  if (!reverse_mode_built(c->p)) {
    c->err = "reverse mode is built for the paper's model only (central-moment fluid, Hall equilibrium, "
             "D3Q27 / D3Q7 velocity sets)";
    return FLAME_E_UNSUPPORTED;
  }
  if (c->p.jmode != FLAME_J_MOMENT || c->p.layout != FLAME_LAYOUT_AA) {
    c->err = "trace step is available on the moment route with the AA layout only";
    return FLAME_E_UNSUPPORTED;
  }
  if (!src || !dst || src == dst) {
    c->err = "trace step needs distinct src and dst";
    return FLAME_E_INVAL;
  }
  const size_t set = 27 * c->n * value_bytes(c->p.storage);
  SetPtrs s{};
  s.f_src = const_cast<void*>(src);
  s.g_src = static_cast<char*>(s.f_src) + set;
  s.f_dst = dst;
  s.g_dst = static_cast<char*>(dst) + set;
  s.fluid_aa = false;
  s.mag_aa = false;
  hipError_t e = launch_step(c, s, c->n, nullptr);
  if (e != hipSuccess) {
    c->err = std::string("step kernel: ") + hipGetErrorString(e);
    return FLAME_E_HIP;
  }
  return FLAME_OK;
}

flame_status flame_adjoint_step(flame_ctx* c, const void* state, const void* lam_next, void* lam, void* lam_j) {
  if (!c) return FLAME_E_INVAL;
  if (!reverse_mode_built(c->p)) {
    c->err = "reverse mode is built for the paper's model only (central-moment fluid, Hall equilibrium, "
             "D3Q27 / D3Q7 velocity sets)";
    return FLAME_E_UNSUPPORTED;
  }
  if (!state || !lam_next || !lam || lam == lam_next || (c->p.jmode == FLAME_J_STENCIL && !lam_j)) {
    c->err = "adjoint step needs state, lam_next and a distinct lam (and lam_j for the stencil route)";
    return FLAME_E_INVAL;
  }
  if (!adjoint_arrays_fit(c)) return FLAME_E_INVAL;
  hipError_t e = c->p.storage == FLAME_F64 ? adjoint_typed<double>(c, state, lam_next, lam, lam_j)
                                           : adjoint_typed<float>(c, state, lam_next, lam, lam_j);
  if (e != hipSuccess) {
    c->err = std::string("adjoint kernel: ") + hipGetErrorString(e);
    return FLAME_E_HIP;
  }
  return FLAME_OK;
}

flame_status flame_adjoint_trace_step(flame_ctx* c, const void* src, const void* lam_next, void* lam) {
  if (!c) return FLAME_E_INVAL;
  if (!reverse_mode_built(c->p)) {
    c->err = "reverse mode is built for the paper's model only (central-moment fluid, Hall equilibrium, "
             "D3Q27 / D3Q7 velocity sets)";
    return FLAME_E_UNSUPPORTED;
  }
  if (c->p.jmode != FLAME_J_MOMENT || c->p.layout != FLAME_LAYOUT_AA) {
    c->err = "the trace adjoint is available on the moment route with the AA layout only";
    return FLAME_E_UNSUPPORTED;
  }
  if (!src || !lam_next || !lam || lam == lam_next) {
    c->err = "trace adjoint needs src, lam_next and a distinct lam";
    return FLAME_E_INVAL;
  }
  if (!adjoint_arrays_fit(c)) return FLAME_E_INVAL;
  hipError_t e;
  switch (c->p.storage) {
    case FLAME_F64: e = adjoint_trace_typed<double>(c, src, lam_next, lam); break;
    case FLAME_F32: e = adjoint_trace_typed<float>(c, src, lam_next, lam); break;
    default: e = adjoint_trace_typed<_Float16>(c, src, lam_next, lam); break;
  }
  if (e != hipSuccess) {
    c->err = std::string("adjoint kernel: ") + hipGetErrorString(e);
    return FLAME_E_HIP;
  }
  return FLAME_OK;
}

flame_status flame_adjoint_init(flame_ctx* c, const void* lam0, const double* u, const double* b,
                                const double* grad_u, const double* grad_b, double* g_u, double* g_b,
                                double* g_grad_u, double* g_grad_b) {
  if (!c) return FLAME_E_INVAL;
  if (!reverse_mode_built(c->p)) {
    c->err = "reverse mode is built for the paper's model only (central-moment fluid, Hall equilibrium, "
             "D3Q27 / D3Q7 velocity sets)";
    return FLAME_E_UNSUPPORTED;
  }
  if (!lam0 || !u || !b || !g_u || !g_b) {
    c->err = "adjoint init needs lam0, u, b, g_u and g_b";
    return FLAME_E_INVAL;
  }
  if (c->p.init_noneq && (!grad_u || !grad_b)) {
    c->err = "adjoint init needs the gradients that flame_init received (the transpose of the "
             "central differences taken in their absence is not built)";
    return FLAME_E_UNSUPPORTED;
  }
  hipError_t e = c->p.storage == FLAME_F64
                     ? init_vjp_typed<double>(c, lam0, u, b, grad_u, grad_b, g_u, g_b, g_grad_u, g_grad_b)
                     : init_vjp_typed<float>(c, lam0, u, b, grad_u, grad_b, g_u, g_b, g_grad_u, g_grad_b);
  if (e != hipSuccess) {
    c->err = std::string("initial-state adjoint kernel: ") + hipGetErrorString(e);
    return FLAME_E_HIP;
  }
  return FLAME_OK;
}

}  // extern "C"
