// The fused time-step kernel: load -> moments -> J -> collide (fluid + magnetic) -> stream.
//
// One thread owns one node. Population sets are stored structure-of-arrays,
// set[q][z][y][x] with x fastest, so a wavefront of 64 threads along x reads and writes
// contiguous 256-byte (FP32) rows per direction. Streaming is done by the addressing:
//   two-lattice (push): read own slots of the source copy, write x + c_i of the other copy;
//   AA in place, even step: read slot i at x, write slot opp(i) at x;
//   AA in place, odd step:  read slot opp(i) at x - c_i, write slot i at x + c_i.
// Each AA thread reads and writes exactly the slots it owns, so the in-place update is
// race-free. With the stencil current the magnetic set is always two-lattice, so the
// neighbour fields read for curl B are never overwritten during the step.

#include "flame_internal.h"

namespace flame {

template <typename S>
struct StepArgs {
  using R = typename Enc<S>::R;
  const S* f_src;
  S* f_dst;
  const S* g_src;
  S* g_dst;
  const R* force_u;   // [3][n] or null
  const R* force_b;   // [3][n] or null
  int nx, ny, nz;
  size_t n;
  PhysConst<R> k;
};

__device__ __forceinline__ size_t node(int x, int y, int z, int nx, int ny) {
  return (static_cast<size_t>(z) * ny + y) * nx + x;
}

// Field fluctuation b_c at a node from the two-lattice (canonical) magnetic source.
template <typename S>
__device__ __forceinline__ typename Enc<S>::R field_at(const StepArgs<S>& a, size_t cell, int comp) {
  using E = Enc<S>;
  using R = typename E::R;
  R s = E::dec(a.g_src[static_cast<size_t>(comp) * a.n + cell], R(1.0 / E::mscale(0)));
#pragma unroll
  for (int i = 1; i < 7; ++i)
    s += E::dec(a.g_src[static_cast<size_t>(i * 3 + comp) * a.n + cell], R(1.0 / E::mscale(i)));
  if (a.force_b) s += R(0.5) * a.force_b[static_cast<size_t>(comp) * a.n + cell];
  return s;
}

// JM: 0 moment route, 1 stencil. FAA / MAA: fluid / magnetic set in place. PAR: AA parity.
template <typename S, int JM, bool FAA, bool MAA, int PAR>
__global__ __launch_bounds__(256) void step_kernel(StepArgs<S> a) {
  using E = Enc<S>;
  using R = typename E::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t n = a.n;
  const size_t cell = node(x, y, z, nx, ny);

  R f[kQ], g[kM];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    size_t src;
    if (FAA && PAR == 1)
      src = static_cast<size_t>(oppq(i)) * n +
            node(wrap(x - cq(i, 0), nx), wrap(y - cq(i, 1), ny), wrap(z - cq(i, 2), nz), nx, ny);
    else
      src = static_cast<size_t>(i) * n + cell;
    f[i] = E::dec(a.f_src[src], R(1.0 / E::fscale(i)));
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      size_t src;
      if (MAA && PAR == 1)
        src = static_cast<size_t>(oppm(i) * 3 + c) * n +
              node(wrap(x - xim(i, 0), nx), wrap(y - xim(i, 1), ny), wrap(z - xim(i, 2), nz), nx, ny);
      else
        src = static_cast<size_t>(i * 3 + c) * n + cell;
      g[i * 3 + c] = E::dec(a.g_src[src], R(1.0 / E::mscale(i)));
    }
  }

  // moments
  const FluidMoments<R> m = fluid_moments(f);
  R F[3] = {R(0), R(0), R(0)}, Sb[3] = {R(0), R(0), R(0)};
  if (a.force_u) {
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] = a.force_u[static_cast<size_t>(c) * n + cell];
  }
  if (a.force_b) {
#pragma unroll
    for (int c = 0; c < 3; ++c) Sb[c] = a.force_b[static_cast<size_t>(c) * n + cell];
  }
  const R rho = R(1) + m.drho;
  const R inv_rho = R(1) / rho;
  const R U[3] = {(m.jx + R(0.5) * F[0]) * inv_rho, (m.jy + R(0.5) * F[1]) * inv_rho,
                  (m.jz + R(0.5) * F[2]) * inv_rho};
  R b[3], lam[3][3];
  magnetic_moments(g, b, lam);
#pragma unroll
  for (int c = 0; c < 3; ++c) b[c] += R(0.5) * Sb[c];
  const R B[3] = {a.k.b0[0] + b[0], a.k.b0[1] + b[1], a.k.b0[2] + b[2]};

  // current density
  R J[3];
  if (JM == 0) {
    current_from_moments(lam, U, B, a.k.alpha, a.k.omega_b, J);
  } else {
    const int xp = wrap(x + 1, nx), xm = wrap(x - 1, nx);
    const int yp = wrap(y + 1, ny), ym = wrap(y - 1, ny);
    const int zp = wrap(z + 1, nz), zm = wrap(z - 1, nz);
    const R bz_yp = field_at(a, node(x, yp, z, nx, ny), 2), bz_ym = field_at(a, node(x, ym, z, nx, ny), 2);
    const R by_zp = field_at(a, node(x, y, zp, nx, ny), 1), by_zm = field_at(a, node(x, y, zm, nx, ny), 1);
    const R bx_zp = field_at(a, node(x, y, zp, nx, ny), 0), bx_zm = field_at(a, node(x, y, zm, nx, ny), 0);
    const R bz_xp = field_at(a, node(xp, y, z, nx, ny), 2), bz_xm = field_at(a, node(xm, y, z, nx, ny), 2);
    const R by_xp = field_at(a, node(xp, y, z, nx, ny), 1), by_xm = field_at(a, node(xm, y, z, nx, ny), 1);
    const R bx_yp = field_at(a, node(x, yp, z, nx, ny), 0), bx_ym = field_at(a, node(x, ym, z, nx, ny), 0);
    J[0] = R(0.5) * (bz_yp - bz_ym) - R(0.5) * (by_zp - by_zm);
    J[1] = R(0.5) * (bx_zp - bx_zm) - R(0.5) * (bz_xp - bz_xm);
    J[2] = R(0.5) * (by_xp - by_xm) - R(0.5) * (bx_yp - bx_ym);
  }

  const R b0[3] = {a.k.b0[0], a.k.b0[1], a.k.b0[2]};
  collide_fluid(f, m, rho, U, b, b0, F, a.k.omega);
  collide_magnetic(g, U, B, b, J, Sb, a.k.alpha, a.k.omega_b);

  // stream + store
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    size_t dst;
    if (FAA && PAR == 0)
      dst = static_cast<size_t>(oppq(i)) * n + cell;
    else
      dst = static_cast<size_t>(i) * n +
            node(wrap(x + cq(i, 0), nx), wrap(y + cq(i, 1), ny), wrap(z + cq(i, 2), nz), nx, ny);
    a.f_dst[dst] = E::enc(f[i], R(E::fscale(i)));
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      size_t dst;
      if (MAA && PAR == 0)
        dst = static_cast<size_t>(oppm(i) * 3 + c) * n + cell;
      else
        dst = static_cast<size_t>(i * 3 + c) * n +
              node(wrap(x + xim(i, 0), nx), wrap(y + xim(i, 1), ny), wrap(z + xim(i, 2), nz), nx, ny);
      a.g_dst[dst] = E::enc(g[i * 3 + c], R(E::mscale(i)));
    }
  }
}

template <typename S>
static hipError_t launch_typed(const flame_ctx* c, const SetPtrs& s) {
  using R = typename Enc<S>::R;
  StepArgs<S> a;
  a.f_src = static_cast<const S*>(s.f_src);
  a.f_dst = static_cast<S*>(s.f_dst);
  a.g_src = static_cast<const S*>(s.g_src);
  a.g_dst = static_cast<S*>(s.g_dst);
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
  const dim3 block(64, 4, 1);
  const dim3 grid((c->p.nx + 63) / 64, (c->p.ny + 3) / 4, c->p.nz);
  const bool st = c->p.jmode == FLAME_J_STENCIL;
  const int par = c->parity;
#define FLAME_LAUNCH(JM, FAA, MAA, PAR) \
  hipLaunchKernelGGL((step_kernel<S, JM, FAA, MAA, PAR>), grid, block, 0, c->stream, a)
  if (!s.fluid_aa) {
    if (st) FLAME_LAUNCH(1, false, false, 0);
    else FLAME_LAUNCH(0, false, false, 0);
  } else if (st) {
    if (par == 0) FLAME_LAUNCH(1, true, false, 0);
    else FLAME_LAUNCH(1, true, false, 1);
  } else {
    if (par == 0) FLAME_LAUNCH(0, true, true, 0);
    else FLAME_LAUNCH(0, true, true, 1);
  }
#undef FLAME_LAUNCH
  return hipGetLastError();
}

hipError_t launch_step(const flame_ctx* c, const SetPtrs& s) {
  switch (c->p.storage) {
    case FLAME_F64: return launch_typed<double>(c, s);
    case FLAME_F32: return launch_typed<float>(c, s);
    default: return launch_typed<_Float16>(c, s);
  }
}

}  // namespace flame
