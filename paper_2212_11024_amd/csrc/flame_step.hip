// The fused time-step kernels: load -> moments -> J -> collide (fluid + magnetic) -> stream.
//
// Population sets are stored structure-of-arrays, set[q][z][y][x] with x fastest, so a
// wavefront of 64 threads along x moves contiguous 256-byte (FP32) rows per direction.
// Streaming is done by the addressing:
//   two-lattice (pull): read slot i at x - c_i of the source copy, write slot i at x of the
//     other copy (all stores aligned);
//   AA in place, even step: read slot i at x, write slot opp(i) at x;
//   AA in place, odd step:  read slot opp(i) at x - c_i, write slot i at x + c_i.
// Each AA thread reads and writes exactly the slots it owns, so the in-place update is
// race-free. With the stencil current the magnetic set is always two-lattice, so the
// neighbour fields read for curl B are never overwritten during the step.
//
// Two kernels:
//   step_local  - moment-route J: every node independent, one node per thread, rows of up to
//     256 nodes per block; with FP16 and FP64 storage its arrays are addressed through buffer
//     resources when every array ends at least 16 bytes below 4 GiB, otherwise (and with FP32
//     storage) through 64-bit global addresses (bitwise the same step either way).
//   step_zmarch - stencil J: a workgroup owns a 64 x 4 tile of (x, y) and marches along z. It
//     keeps the field fluctuation b of three consecutive planes in LDS (computed once per node
//     from that node's own magnetic populations, which it holds in registers for the next
//     iteration) plus, for each plane, the one-node ring around the tile (computed one plane
//     ahead); J is the central-difference curl read from LDS.

#include <algorithm>

#include "flame_access.h"
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
  int zchunk;         // planes per workgroup (z-marching kernel)
  size_t n;           // nodes (stride of the caller's forcing arrays)
  size_t stride;      // elements between consecutive population arrays (n plus padding)
  R* save;            // optional: pre-collision state [48 populations + 3 J][n] of this step
  PhysConst<R> k;
};

// Stencil kernel: compute the ring of b around the tile one plane ahead, together with the
// tile's own loads of that plane (the ring nodes' populations are the ones the neighbouring
// tiles load at about the same time); 0 computes it for the current plane.
#ifndef FLAME_ZMARCH_RING_AHEAD
#define FLAME_ZMARCH_RING_AHEAD 1
#endif

// Fluid populations of the node. FAA: in place (PAR selects the AA step); else pull.
template <typename S, bool FAA, int PAR, Addr A = Addr::Global>
__device__ __forceinline__ void load_fluid(const StepArgs<S>& a, const Rows& rw, const Planes& pl,
                                           typename Enc<S>::R (&f)[kQ]) {
  using E = Enc<S>;
  using R = typename E::R;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const bool own = FAA && PAR == 0;
    const uint32_t off = own ? rw.at(0, 0) + pl.at(0) : rw.at(-cq(i, 0), -cq(i, 1)) + pl.at(-cq(i, 2));
    const S* base = a.f_src + static_cast<size_t>(FAA && PAR == 1 ? oppq(i) : i) * a.stride;
    f[i] = E::dec(ld<A>(base, off), R(1.0 / E::fscale(i)));
  }
}

template <typename S, bool FAA, int PAR, Addr A = Addr::Global>
__device__ __forceinline__ void store_fluid(const StepArgs<S>& a, const Rows& rw, const Planes& pl,
                                            const typename Enc<S>::R (&f)[kQ]) {
  using E = Enc<S>;
  using R = typename E::R;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const bool shifted = FAA && PAR == 1;
    const uint32_t off = shifted ? rw.at(cq(i, 0), cq(i, 1)) + pl.at(cq(i, 2)) : rw.at(0, 0) + pl.at(0);
    S* base = a.f_dst + static_cast<size_t>(FAA && PAR == 0 ? oppq(i) : i) * a.stride;
    st<A>(base, off, E::enc(f[i], R(E::fscale(i))));
  }
}

template <typename S, bool MAA, int PAR, Addr A = Addr::Global>
__device__ __forceinline__ void load_magnetic(const StepArgs<S>& a, const Rows& rw, const Planes& pl,
                                              typename Enc<S>::R (&g)[kM]) {
  using E = Enc<S>;
  using R = typename E::R;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const bool own = MAA && PAR == 0;
    const uint32_t off = own ? rw.at(0, 0) + pl.at(0) : rw.at(-xim(i, 0), -xim(i, 1)) + pl.at(-xim(i, 2));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const S* base = a.g_src + static_cast<size_t>((MAA && PAR == 1 ? oppm(i) : i) * 3 + c) * a.stride;
      g[i * 3 + c] = E::dec(ld<A>(base, off), R(1.0 / E::mscale(i)));
    }
  }
}

template <typename S, bool MAA, int PAR, Addr A = Addr::Global>
__device__ __forceinline__ void store_magnetic(const StepArgs<S>& a, const Rows& rw, const Planes& pl,
                                               const typename Enc<S>::R (&g)[kM]) {
  using E = Enc<S>;
  using R = typename E::R;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const bool shifted = MAA && PAR == 1;
    const uint32_t off = shifted ? rw.at(xim(i, 0), xim(i, 1)) + pl.at(xim(i, 2)) : rw.at(0, 0) + pl.at(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      S* base = a.g_dst + static_cast<size_t>((MAA && PAR == 0 ? oppm(i) : i) * 3 + c) * a.stride;
      st<A>(base, off, E::enc(g[i * 3 + c], R(E::mscale(i))));
    }
  }
}

template <typename S, Addr A = Addr::Global>
__device__ __forceinline__ void forcing_at(const StepArgs<S>& a, uint32_t cell, typename Enc<S>::R (&F)[3],
                                           typename Enc<S>::R (&Sb)[3]) {
  using R = typename Enc<S>::R;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    F[c] = a.force_u ? ld<A>(a.force_u + static_cast<size_t>(c) * a.n, cell) : R(0);
    Sb[c] = a.force_b ? ld<A>(a.force_b + static_cast<size_t>(c) * a.n, cell) : R(0);
  }
}

// Model variants, chosen at compile time (0 is the paper's scheme): bit kModelBGK, the BGK fluid
// collision (S = omega I); bit kModelEMHD, electron MHD (the magnetic equilibrium and the J
// system see a zero bulk velocity).
constexpr int kModelBGK = 1;
constexpr int kModelEMHD = 2;

template <typename R>
struct Zero3 {
  R v[3] = {R(0), R(0), R(0)};
};

// Fluid collision of the model, in place.
template <int MODEL, bool Grouped, typename R>
__device__ __forceinline__ void collide_fluid_model(R (&f)[kQ], const FluidMoments<R>& m, const R (&U)[3],
                                                    const R (&b)[3], const R (&b0)[3], const R (&F)[3], R omega) {
  if constexpr ((MODEL & kModelBGK) != 0)
    collide_fluid_bgk(f, m, U, b, b0, F, omega);
  else
    collide_fluid<R, Grouped>(f, m, R(1) + m.drho, U, b, b0, F, omega);
}

// Node update from loaded populations and J: moments, both collisions, in place in f and g.
// Um is the bulk velocity as the magnetic equilibrium sees it (zero for electron MHD).
template <int MODEL, bool Grouped, typename R>
__device__ __forceinline__ void collide_node(R (&f)[kQ], R (&g)[kM], const FluidMoments<R>& m, const R (&U)[3],
                                             const R (&Um)[3], const R (&b)[3], const R (&J)[3], const R (&F)[3],
                                             const R (&Sb)[3], const PhysConst<R>& k) {
  const R b0[3] = {k.b0[0], k.b0[1], k.b0[2]};
  const R B[3] = {b0[0] + b[0], b0[1] + b[1], b0[2] + b[2]};
  collide_fluid_model<MODEL, Grouped>(f, m, U, b, b0, F, k.omega);
  collide_magnetic(g, Um, B, b, J, Sb, k.alpha, k.omega_b);
}

// Record the node's pre-collision deviations (and the J it uses) for the adjoint (streamed out
// with the step's own addressing and store hint; read back only by the reverse sweep).
template <Addr A, typename R>
__device__ __forceinline__ void save_state(R* save, size_t n, uint32_t cell, const R (&f)[kQ], const R (&g)[kM]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) st<A>(save + static_cast<size_t>(q) * n, cell, f[q]);
#pragma unroll
  for (int q = 0; q < kM; ++q) st<A>(save + static_cast<size_t>(kQ + q) * n, cell, g[q]);
}
template <Addr A, typename R>
__device__ __forceinline__ void save_current(R* save, size_t n, uint32_t cell, const R (&J)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) st<A>(save + static_cast<size_t>(kQ + kM + c) * n, cell, J[c]);
}

// ------------------------------------------------------------------ moment-route kernel
constexpr int kLocalThreads = 256;
static_assert(kLocalThreads == kRowThreadsMax, "row blocks are launched with up to kRowThreadsMax threads");

template <typename S, bool FAA, bool MAA, int PAR, bool SAVE, int MODEL, Addr A>
__global__ __launch_bounds__(kLocalThreads) void step_local(StepArgs<S> a) {
  using R = typename Enc<S>::R;
  unsigned bx, by, bz;
  logical_block((a.nx + blockDim.x - 1) / blockDim.x, a.ny, a.nz, bx, by, bz);
  const int x = bx * blockDim.x + threadIdx.x;
  const int y = by;
  const int z = bz;
  if (x >= a.nx) return;
  const Rows rw(x, y, a.nx, a.ny);
  const Planes pl(z, a.nz, static_cast<uint32_t>(a.nx) * a.ny);
  const uint32_t cell = rw.at(0, 0) + pl.at(0);
  R f[kQ], g[kM];
  load_fluid<S, FAA, PAR, A>(a, rw, pl, f);
  load_magnetic<S, MAA, PAR, A>(a, rw, pl, g);
  R F[3], Sb[3];
  forcing_at<S, A>(a, cell, F, Sb);
  if (SAVE) save_state<A>(a.save, a.n, cell, f, g);
  const FluidMoments<R> m = fluid_moments(f);
  const R inv_rho = R(1) / (R(1) + m.drho);
  const R U[3] = {(m.jx + R(0.5) * F[0]) * inv_rho, (m.jy + R(0.5) * F[1]) * inv_rho,
                  (m.jz + R(0.5) * F[2]) * inv_rho};
  R b[3], lam[3][3];
  magnetic_moments(g, b, lam);
#pragma unroll
  for (int c = 0; c < 3; ++c) b[c] = b_component(g, c, R(0.5) * Sb[c]);
  const R B[3] = {a.k.b0[0] + b[0], a.k.b0[1] + b[1], a.k.b0[2] + b[2]};
  const Zero3<R> zero;
  const R(&Um)[3] = (MODEL & kModelEMHD) != 0 ? zero.v : U;
  R J[3];
  current_from_moments(lam, Um, B, a.k.alpha, a.k.omega_b, J);
  if (SAVE) save_current<A>(a.save, a.n, cell, J);
  collide_node<MODEL, sizeof(S) == 2>(f, g, m, U, Um, b, J, F, Sb, a.k);
  store_fluid<S, FAA, PAR, A>(a, rw, pl, f);
  store_magnetic<S, MAA, PAR, A>(a, rw, pl, g);
}

// ------------------------------------------------------------------ stencil-route kernel
// Tile and z-chunk of the stencil kernel (tuning parameters, overridable at build time).
#ifndef FLAME_TY
#define FLAME_TY 4        // FP32 / FP16 storage
#endif
#ifndef FLAME_TY64
#define FLAME_TY64 4      // FP64 storage (twice the registers per node)
#endif
#ifndef FLAME_ZCHUNK
#define FLAME_ZCHUNK 32
#endif
#ifndef FLAME_ZMARCH_WAVES_PER_EU
#define FLAME_ZMARCH_WAVES_PER_EU 1
#endif
constexpr int kTX = 64;
template <typename R>
struct Tile {
  static constexpr int ty = sizeof(R) == 8 ? FLAME_TY64 : FLAME_TY;
};
constexpr int kZChunk = FLAME_ZCHUNK;   // planes per workgroup

template <typename S, bool FAA, int PAR, bool SAVE, int MODEL>
__global__ __launch_bounds__(kTX * Tile<typename Enc<S>::R>::ty, FLAME_ZMARCH_WAVES_PER_EU) void step_zmarch(
    StepArgs<S> a) {
  using E = Enc<S>;
  using R = typename E::R;
  constexpr int kTY = Tile<R>::ty;
  // b of the tile plus its one-node ring for a rolling window of planes:
  // [plane slot][ly + 1][lx + 1][component]. Four slots: a slot is rewritten two iterations
  // after it was last read, so one barrier per plane separates every write from every read.
  __shared__ R sb[4][kTY + 2][kTX + 2][3];
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  unsigned bx, by, bz;
  logical_block((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY, (nz + a.zchunk - 1) / a.zchunk, bx, by, bz);
  const int x0 = bx * kTX, y0 = by * kTY;
  const int w = min(kTX, nx - x0), h = min(kTY, ny - y0);
  const int z_begin = bz * a.zchunk;
  const int z_end = min(nz, z_begin + a.zchunk);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int tid = ly * kTX + lx;
  const bool active = lx < w && ly < h;
  const int x = x0 + lx, y = y0 + ly;

  const uint32_t plane = static_cast<uint32_t>(nx) * ny;
  const Rows rw(active ? x : 0, active ? y : 0, nx, ny);
  auto half_src = [&](uint32_t cell, int c) -> R {
    return a.force_b ? R(0.5) * ld<Addr::Global>(a.force_b + static_cast<size_t>(c) * a.n, cell) : R(0);
  };
  auto put_b = [&](int slot, const R (&g)[kM], uint32_t cell) {
#pragma unroll
    for (int c = 0; c < 3; ++c) sb[slot][ly + 1][lx + 1][c] = b_component(g, c, half_src(cell, c));
  };
  // ring nodes of a plane: two components of b from their seven pulled populations
  auto ring = [&](int slot, const Planes& pl) {
    for (int task = tid; task < 2 * w + 2 * h; task += kTX * kTY) {
      int rx, ry, c0, c1;
      if (task < 2 * w) {
        rx = task < w ? task : task - w;
        ry = task < w ? -1 : h;
        c0 = 0; c1 = 2;                       // y-neighbours enter through B_x and B_z
      } else {
        const int t = task - 2 * w;
        ry = t < h ? t : t - h;
        rx = t < h ? -1 : w;
        c0 = 1; c1 = 2;                       // x-neighbours enter through B_y and B_z
      }
      const Rows rr(wrap(x0 + rx, nx), wrap(y0 + ry, ny), nx, ny);
      // same summation order as b_component
      R s0 = R(0), s1 = R(0);
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const uint32_t off = rr.at(-xim(i, 0), -xim(i, 1)) + pl.at(-xim(i, 2));
        const R v0 =
            E::dec(ld<Addr::Global>(a.g_src + static_cast<size_t>(i * 3 + c0) * a.stride, off), R(1.0 / E::mscale(i)));
        const R v1 =
            E::dec(ld<Addr::Global>(a.g_src + static_cast<size_t>(i * 3 + c1) * a.stride, off), R(1.0 / E::mscale(i)));
        s0 = i == 0 ? v0 : s0 + v0;
        s1 = i == 0 ? v1 : s1 + v1;
      }
      const uint32_t cell = rr.at(0, 0) + pl.at(0);
      sb[slot][ry + 1][rx + 1][c0] = s0 + half_src(cell, c0);
      sb[slot][ry + 1][rx + 1][c1] = s1 + half_src(cell, c1);
    }
  };

  R g_next[kM];
  const Planes p0(z_begin, nz, plane);
  if (active) {
    R gp[kM];
    const Planes pp(wrap(z_begin - 1, nz), nz, plane);
    load_magnetic<S, false, 0>(a, rw, pp, gp);
    put_b(0, gp, rw.at(0, 0) + pp.at(0));
    load_magnetic<S, false, 0>(a, rw, p0, g_next);
    put_b(1, g_next, rw.at(0, 0) + p0.at(0));
  }
  if (FLAME_ZMARCH_RING_AHEAD) ring(1, p0);
  int prev = 0, cur = 1, next = 2, spare = 3;
  for (int z = z_begin; z < z_end; ++z) {
    R g[kM];
#pragma unroll
    for (int q = 0; q < kM; ++q) g[q] = g_next[q];
    const Planes pl(z, nz, plane);
    const Planes pn(wrap(z + 1, nz), nz, plane);
    const uint32_t cell = rw.at(0, 0) + pl.at(0);
    R U[3], b[3], F[3], Sb[3];
    if (active) {
      load_magnetic<S, false, 0>(a, rw, pn, g_next);
      put_b(next, g_next, rw.at(0, 0) + pn.at(0));
    }
    if (FLAME_ZMARCH_RING_AHEAD)
      ring(next, pn);
    else
      ring(cur, pl);
    if (active) {
      // the fluid half of the update needs no J: collide and store it before the barrier
      R f[kQ];
      load_fluid<S, FAA, PAR>(a, rw, pl, f);
      forcing_at(a, cell, F, Sb);
      if (SAVE) save_state<Addr::Global>(a.save, a.n, cell, f, g);
      const FluidMoments<R> m = fluid_moments(f);
      const R inv_rho = R(1) / (R(1) + m.drho);
      U[0] = (m.jx + R(0.5) * F[0]) * inv_rho;
      U[1] = (m.jy + R(0.5) * F[1]) * inv_rho;
      U[2] = (m.jz + R(0.5) * F[2]) * inv_rho;
#pragma unroll
      for (int c = 0; c < 3; ++c) b[c] = b_component(g, c, R(0.5) * Sb[c]);
      const R b0[3] = {a.k.b0[0], a.k.b0[1], a.k.b0[2]};
      collide_fluid_model<MODEL, false>(f, m, U, b, b0, F, a.k.omega);
      store_fluid<S, FAA, PAR>(a, rw, pl, f);
    }
    __syncthreads();
    if (active) {
      const R(&P)[kTY + 2][kTX + 2][3] = sb[prev];
      const R(&C)[kTY + 2][kTX + 2][3] = sb[cur];
      const R(&N)[kTY + 2][kTX + 2][3] = sb[next];
      const int px = lx + 1, py = ly + 1;
      R J[3];
      J[0] = R(0.5) * (C[py + 1][px][2] - C[py - 1][px][2]) - R(0.5) * (N[py][px][1] - P[py][px][1]);
      J[1] = R(0.5) * (N[py][px][0] - P[py][px][0]) - R(0.5) * (C[py][px + 1][2] - C[py][px - 1][2]);
      J[2] = R(0.5) * (C[py][px + 1][1] - C[py][px - 1][1]) - R(0.5) * (C[py + 1][px][0] - C[py - 1][px][0]);
      const R B[3] = {a.k.b0[0] + b[0], a.k.b0[1] + b[1], a.k.b0[2] + b[2]};
      if (SAVE) save_current<Addr::Global>(a.save, a.n, cell, J);
      const Zero3<R> zero;
      collide_magnetic(g, (MODEL & kModelEMHD) != 0 ? zero.v : U, B, b, J, Sb, a.k.alpha, a.k.omega_b);
      store_magnetic<S, false, 0>(a, rw, pl, g);
    }
    const int t = prev;
    prev = cur;
    cur = next;
    next = spare;
    spare = t;
  }
}

template <typename S, bool SAVE, int MODEL, Addr A>
static void launch_local(const flame_ctx* c, const SetPtrs& s, const StepArgs<S>& a) {
  const unsigned tx = row_threads(c);
  const dim3 block(tx, 1, 1);
  const dim3 grid(((c->p.nx + tx - 1) / tx) * c->p.ny * c->p.nz);
  if (!s.fluid_aa)
    hipLaunchKernelGGL((step_local<S, false, false, 0, SAVE, MODEL, A>), grid, block, 0, c->stream, a);
  else if (c->parity == 0)
    hipLaunchKernelGGL((step_local<S, true, true, 0, SAVE, MODEL, A>), grid, block, 0, c->stream, a);
  else
    hipLaunchKernelGGL((step_local<S, true, true, 1, SAVE, MODEL, A>), grid, block, 0, c->stream, a);
}

template <typename S, bool SAVE, int MODEL>
static void launch_model(const flame_ctx* c, const SetPtrs& s, const StepArgs<S>& a) {
  using R = typename Enc<S>::R;
  const int par = c->parity;
  if (c->p.jmode == FLAME_J_STENCIL) {
    constexpr int kTY = Tile<R>::ty;
    const dim3 grid(((c->p.nx + kTX - 1) / kTX) * ((c->p.ny + kTY - 1) / kTY) * ((c->p.nz + a.zchunk - 1) / a.zchunk));
    const dim3 block(kTX, kTY, 1);
    if (!s.fluid_aa)
      hipLaunchKernelGGL((step_zmarch<S, false, 0, SAVE, MODEL>), grid, block, 0, c->stream, a);
    else if (par == 0)
      hipLaunchKernelGGL((step_zmarch<S, true, 0, SAVE, MODEL>), grid, block, 0, c->stream, a);
    else
      hipLaunchKernelGGL((step_zmarch<S, true, 1, SAVE, MODEL>), grid, block, 0, c->stream, a);
  } else {
    // FP16 and FP64 storage: buffer resources (timed on the same buffers at 512^3, FP16 6.05-6.12
    // against 6.43-6.50 ms, FP64 18.91-19.13 against 19.17-19.30 ms); FP32 keeps the global
    // addresses, with which it runs 1.1-2.5% faster (9.09 against 9.20 ms on a fast placement)
    if constexpr (sizeof(S) != 4) {
      const bool arith_arrays = SAVE || c->p.force_u || c->p.force_b;
      if (!c->global_addr && buffer_addressing_ok(c->p, arith_arrays)) {
        launch_local<S, SAVE, MODEL, Addr::Buffer>(c, s, a);
        return;
      }
    }
    launch_local<S, SAVE, MODEL, Addr::Global>(c, s, a);
  }
}

template <typename S, bool SAVE>
static hipError_t launch_typed(const flame_ctx* c, const SetPtrs& s, size_t stride, void* save) {
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
  a.stride = stride;
  a.save = static_cast<R*>(save);
  a.k.omega = R(c->omega);
  a.k.omega_b = R(c->omega_b);
  a.k.alpha = R(c->p.d_i);
  for (int i = 0; i < 3; ++i) a.k.b0[i] = R(c->p.b0[i]);
  a.zchunk = c->p.jmode == FLAME_J_STENCIL ? std::min(c->p.nz, c->zchunk > 0 ? c->zchunk : kZChunk) : 1;
  const int model = step_model(c->p);
  if constexpr (SAVE) {
    // the state-saving steps serve the adjoint, which is built for the paper's model only
    if (model != 0) return hipErrorInvalidValue;
    launch_model<S, true, 0>(c, s, a);
  } else {
    switch (model) {
      case 0: launch_model<S, false, 0>(c, s, a); break;
      case kModelBGK: launch_model<S, false, kModelBGK>(c, s, a); break;
      case kModelEMHD: launch_model<S, false, kModelEMHD>(c, s, a); break;
      default: launch_model<S, false, kModelBGK | kModelEMHD>(c, s, a); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_step(const flame_ctx* c, const SetPtrs& s, size_t stride, void* save) {
  if (lattice_variant(c->p)) return save ? hipErrorInvalidValue : variant_launch_step(c, s);
  switch (c->p.storage) {
    case FLAME_F64:
      return save ? launch_typed<double, true>(c, s, stride, save) : launch_typed<double, false>(c, s, stride, save);
    case FLAME_F32:
      return save ? launch_typed<float, true>(c, s, stride, save) : launch_typed<float, false>(c, s, stride, save);
    default:
      return save ? launch_typed<_Float16, true>(c, s, stride, save)
                  : launch_typed<_Float16, false>(c, s, stride, save);
  }
}

}  // namespace flame
