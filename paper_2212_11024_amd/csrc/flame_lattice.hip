// Lattice variants of the step: the D3Q19 fluid set and the D3Q15 / D3Q27 magnetic sets (the
// lattice figure of Sec. 3.1; Sec. 4.3 reports runs with the larger magnetic sets), on the moment
// route of J. The paper's pair (D3Q27 fluid, D3Q7 magnetic) keeps its own kernels
// (flame_step.hip, flame_api.hip); this file serves every other pair, with the same storage
// encodings, layouts (AA in place for both sets, or two lattices with pull streaming), canonical
// ordering rules and FP64 diagnostics:
//   - a node-local fused step (one node per thread, rows of up to 256 nodes per block);
//   - the initial state, canonical copies, node fields, reduction partials and the field
//     components the spectra transform.
// Readings the paper leaves open (velocity orders, magnetic weights, the D3Q19 equilibrium and
// force term) are stated in include/flame.h next to the FLAME_FLUID_* / FLAME_MAGNETIC_* values.

#include <math.h>

#include "flame_internal.h"
#include "flame_lattice.h"

namespace flame {
namespace lattice {

// ------------------------------------------------------------------ addressing
__device__ __forceinline__ size_t vnode(int x, int y, int z, int nx, int ny) {
  return (static_cast<size_t>(z) * ny + y) * nx + x;
}
__device__ __forceinline__ void vxyz(size_t cell, int nx, int ny, int& x, int& y, int& z) {
  x = static_cast<int>(cell % nx);
  const size_t r = cell / nx;
  y = static_cast<int>(r % ny);
  z = static_cast<int>(r / ny);
}

// Where a step or a reader finds canonical population i (velocity v) of node (x, y, z) in a set:
// mode 0: slot i at x (AA even step); 1: slot opp(i) at x - v (AA odd step); 2: slot i at x - v
// (two-lattice pull source).
struct SetGeom {
  int nx, ny, nz;
  size_t stride;
  // the slot and the node of that population
  __device__ int slot(int mode, int i, int opp) const { return mode == 1 ? opp : i; }
  __device__ size_t node(int mode, int vx, int vy, int vz, int x, int y, int z) const {
    if (mode == 0) return vnode(x, y, z, nx, ny);
    return vnode(wrap(x - vx, nx), wrap(y - vy, ny), wrap(z - vz, nz), nx, ny);
  }
  __device__ size_t at(int mode, int i, int opp, int vx, int vy, int vz, int x, int y, int z) const {
    return static_cast<size_t>(slot(mode, i, opp)) * stride + node(mode, vx, vy, vz, x, y, z);
  }
};

// ------------------------------------------------------------------ fused step
template <typename S>
struct VStepArgs {
  using R = typename Enc<S>::R;
  const S* f_src;
  S* f_dst;
  const S* g_src;
  S* g_dst;
  const R* force_u;
  const R* force_b;
  int nx, ny, nz;
  size_t n, stride;
  PhysConst<R> k;
};

// AA: both sets in place (PAR: even 0 / odd 1); else two-lattice pull for both.
template <typename S, typename FL, typename ML, bool AA, int PAR, bool BGK, bool EMHD>
__global__ __launch_bounds__(256) void variant_step(VStepArgs<S> a) {
  using E = Enc<S>;
  using R = typename E::R;
  constexpr int Q = FL::q, NG = ML::m * 3;
  unsigned bx, by, bz;
  logical_block((a.nx + blockDim.x - 1) / blockDim.x, a.ny, a.nz, bx, by, bz);
  const int x = bx * blockDim.x + threadIdx.x, y = by, z = bz;
  if (x >= a.nx) return;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t cell = vnode(x, y, z, nx, ny);
  const SetGeom geo{nx, ny, nz, a.stride};
  const int rmode = AA ? PAR : 2;
  R f[Q], g[NG];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    f[i] = E::dec(a.f_src[geo.at(rmode, i, FL::opp(i), FL::c(i, 0), FL::c(i, 1), FL::c(i, 2), x, y, z)],
                  R(1.0 / fscale<S, FL>(i)));
#pragma unroll
  for (int i = 0; i < ML::m; ++i) {
    const size_t slot = geo.slot(rmode, i, ML::opp(i));
    const size_t node = geo.node(rmode, ML::xi(i, 0), ML::xi(i, 1), ML::xi(i, 2), x, y, z);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      g[i * 3 + c] = E::dec(a.g_src[(slot * 3 + c) * a.stride + node], R(1.0 / fscale<S, ML>(i)));
  }
  R F[3], Sb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    F[c] = a.force_u ? a.force_u[static_cast<size_t>(c) * a.n + cell] : R(0);
    Sb[c] = a.force_b ? a.force_b[static_cast<size_t>(c) * a.n + cell] : R(0);
  }
  variant_node<FL, ML, BGK, EMHD>(f, g, F, Sb, a.k);
  // stores: AA even: slot opp(i) at x; AA odd: slot i at x + v; pull: slot i at x (other copy)
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    size_t idx;
    if (AA && PAR == 0) idx = static_cast<size_t>(FL::opp(i)) * a.stride + cell;
    else if (AA) idx = static_cast<size_t>(i) * a.stride + vnode(wrap(x + FL::c(i, 0), nx), wrap(y + FL::c(i, 1), ny),
                                                             wrap(z + FL::c(i, 2), nz), nx, ny);
    else idx = static_cast<size_t>(i) * a.stride + cell;
    a.f_dst[idx] = E::enc(f[i], R(fscale<S, FL>(i)));
  }
#pragma unroll
  for (int i = 0; i < ML::m; ++i) {
    size_t slot, node;
    if (AA && PAR == 0) { slot = ML::opp(i); node = cell; }
    else if (AA) { slot = i; node = vnode(wrap(x + ML::xi(i, 0), nx), wrap(y + ML::xi(i, 1), ny), wrap(z + ML::xi(i, 2), nz), nx, ny); }
    else { slot = i; node = cell; }
#pragma unroll
    for (int c = 0; c < 3; ++c)
      a.g_dst[(slot * 3 + c) * a.stride + node] = E::enc(g[i * 3 + c], R(fscale<S, ML>(i)));
  }
}

// ------------------------------------------------------------------ canonical view
template <typename S, typename FL, typename ML>
struct VView {
  const S* F;
  const S* G;
  int fmode, gmode;
  SetGeom geo;
  size_t n;
  __device__ double f(int i, int x, int y, int z) const {
    return static_cast<double>(F[geo.at(fmode, i, FL::opp(i), FL::c(i, 0), FL::c(i, 1), FL::c(i, 2), x, y, z)]) /
           fscale<S, FL>(i);
  }
  __device__ double g(int i, int c, int x, int y, int z) const {
    const size_t slot = geo.slot(gmode, i, ML::opp(i));
    const size_t node = geo.node(gmode, ML::xi(i, 0), ML::xi(i, 1), ML::xi(i, 2), x, y, z);
    return static_cast<double>(G[(slot * 3 + c) * geo.stride + node]) / fscale<S, ML>(i);
  }
};

template <typename S, typename FL, typename ML>
struct VAux {
  VView<S, FL, ML> v;
  const typename Enc<S>::R* force_u;
  const typename Enc<S>::R* force_b;
  double b0[3];
  double alpha, omega_b;
  int emhd;
};

// Node quantities of the current state in FP64: rho, U, B (with the forcing half-shifts), b, J
// (moment route), div B estimate, finiteness.
template <typename S, typename FL, typename ML>
__device__ void node_q(const VAux<S, FL, ML>& a, int x, int y, int z, double& rho, double (&U)[3], double (&B)[3],
                       double (&b)[3], double (&J)[3], double& divb, bool& finite) {
  const size_t cell = vnode(x, y, z, a.v.geo.nx, a.v.geo.ny);
  // unrolled, so that g stays in registers (a runtime index would put it in per-thread private memory)
  double g[ML::m * 3];
  bool fin = true;
  double drho = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < FL::q; ++i) {
    const double fi = a.v.f(i, x, y, z);
    fin = fin && isfinite(fi);
    drho += fi;
#pragma unroll
    for (int c = 0; c < 3; ++c) j[c] += FL::c(i, c) * fi;
  }
#pragma unroll
  for (int i = 0; i < ML::m; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[i * 3 + c] = a.v.g(i, c, x, y, z);
      fin = fin && isfinite(g[i * 3 + c]);
    }
  finite = fin;
  rho = 1.0 + drho;
  const size_t n = a.v.n;
  for (int c = 0; c < 3; ++c) {
    const double F = a.force_u ? static_cast<double>(a.force_u[c * n + cell]) : 0.0;
    U[c] = (j[c] + 0.5 * F) / rho;
  }
  double lam[3][3];
  mag_moments<ML>(g, b, lam);
  for (int c = 0; c < 3; ++c) {
    const double src = a.force_b ? static_cast<double>(a.force_b[c * n + cell]) : 0.0;
    b[c] += 0.5 * src;
    B[c] = a.b0[c] + b[c];
  }
  const double zero[3] = {0.0, 0.0, 0.0};
  current_from_moments(lam, a.emhd ? zero : U, B, a.alpha, a.omega_b, J);
  divb = -4.0 * a.omega_b * (lam[0][0] + lam[1][1] + lam[2][2]);
}

// ------------------------------------------------------------------ initial state
template <typename S>
struct VInitArgs {
  using R = typename Enc<S>::R;
  S* F;
  S* G;
  const double* u;
  const double* b;
  const double* gu;
  const double* gb;
  const R* force_u;
  const R* force_b;
  double b0[3];
  double omega, omega_b, alpha;
  int noneq, emhd;
  int nx, ny, nz;
  size_t n, stride;
  int fpull, gpull;   // write population i at x - v (two-lattice pull source) instead of x
};

template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(256) void variant_init(VInitArgs<S> a) {
  using E = Enc<S>;
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.n) return;
  const size_t n = a.n;
  int px, py, pz;
  vxyz(cell, a.nx, a.ny, px, py, pz);
  double U[3], b[3], B[3], F[3] = {0, 0, 0}, Sb[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) {
    U[c] = a.u[c * n + cell];
    b[c] = a.b[c * n + cell];
    B[c] = a.b0[c] + b[c];
    if (a.force_u) F[c] = static_cast<double>(a.force_u[c * n + cell]);
    if (a.force_b) Sb[c] = static_cast<double>(a.force_b[c * n + cell]);
  }
  auto central = [&](const double* v, double (&g)[3][3]) {
    const size_t xm = vnode(wrap(px - 1, a.nx), py, pz, a.nx, a.ny), xp = vnode(wrap(px + 1, a.nx), py, pz, a.nx, a.ny);
    const size_t ym = vnode(px, wrap(py - 1, a.ny), pz, a.nx, a.ny), yp = vnode(px, wrap(py + 1, a.ny), pz, a.nx, a.ny);
    const size_t zm = vnode(px, py, wrap(pz - 1, a.nz), a.nx, a.ny), zp = vnode(px, py, wrap(pz + 1, a.nz), a.nx, a.ny);
    for (int c = 0; c < 3; ++c) {
      const double* vc = v + c * n;
      g[0][c] = 0.5 * (vc[xp] - vc[xm]);
      g[1][c] = 0.5 * (vc[yp] - vc[ym]);
      g[2][c] = 0.5 * (vc[zp] - vc[zm]);
    }
  };
  double G[3][3] = {}, H[3][3] = {};
  bool have_gu = a.gu != nullptr, have_gb = a.gb != nullptr;
  if (a.gu) {
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) G[p][q] = a.gu[(p * 3 + q) * n + cell];
  } else if (a.noneq) {
    central(a.u, G);
    have_gu = true;
  }
  if (a.gb) {
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) H[p][q] = a.gb[(p * 3 + q) * n + cell];
  } else if (a.noneq) {
    central(a.b, H);
    have_gb = true;
  }
  // fluid
  double f[FL::q];
  if constexpr (FL::q == 27) {
    PhysConst<double> k;
    k.omega = a.omega;
    k.omega_b = a.omega_b;
    k.alpha = a.alpha;
    for (int c = 0; c < 3; ++c) k.b0[c] = a.b0[c];
    InitFlags fl;
    fl.fluid_noneq = a.noneq && have_gu;
    fl.mag_noneq = false;
    fl.has_H = false;
    fl.emhd = false;
    double g7[kM];
    init_node(U, b, G, H, F, Sb, k, fl, f, g7);   // its D3Q27 fluid part
  } else {
    double P[3][3] = {};
    if (a.noneq && have_gu) {
      const double div = G[0][0] + G[1][1] + G[2][2];
      const double s = -(1.0 / 3.0) / a.omega;
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) P[p][q] = s * (G[p][q] + G[q][p] - (p == q ? 2.0 / 3.0 * div : 0.0));
    }
    const double u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const double sb = a.b0[0] * b[0] + a.b0[1] * b[1] + a.b0[2] * b[2] + 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double b0[3] = {a.b0[0], a.b0[1], a.b0[2]};
    for (int i = 0; i < FL::q; ++i) {
      double v = eq2_deviation<FL>(i, 0.0, U, u2, sb, b, b0);
      // (w / 2 c_s^4) P : (c c - c_s^2 I); P is traceless
      double pc = 0;
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) pc += P[p][q] * FL::c(i, p) * FL::c(i, q);
      v += FL::w(i) * 4.5 * pc;
      v -= 0.5 * force2<FL>(i, U, F);
      f[i] = v;
    }
  }
  // magnetic: W_i (b + 4 xi.(V B - B V)) - (1 / w_B) W_i xi_p H_pc - S/2 W_i
  double J[3] = {0, 0, 0};
  if (have_gb) {
    J[0] = H[1][2] - H[2][1];
    J[1] = H[2][0] - H[0][2];
    J[2] = H[0][1] - H[1][0];
  }
  const double um = a.emhd ? 0.0 : 1.0;
  const double V[3] = {um * U[0] - a.alpha * J[0], um * U[1] - a.alpha * J[1], um * U[2] - a.alpha * J[2]};
  const bool mag_noneq = a.noneq && have_gb;
  for (int i = 0; i < ML::m; ++i) {
    size_t gnode = cell;
    if (a.gpull)
      gnode = vnode(wrap(px - ML::xi(i, 0), a.nx), wrap(py - ML::xi(i, 1), a.ny), wrap(pz - ML::xi(i, 2), a.nz), a.nx, a.ny);
    for (int c = 0; c < 3; ++c) {
      double xv = 0, xb = 0, xg = 0;
      for (int p = 0; p < 3; ++p) {
        xv += ML::xi(i, p) * V[p];
        xb += ML::xi(i, p) * B[p];
        xg += ML::xi(i, p) * H[p][c];
      }
      double v = ML::w(i) * (b[c] + 4.0 * (xv * B[c] - xb * V[c]));
      if (mag_noneq) v -= ML::w(i) * xg / a.omega_b;
      v -= 0.5 * ML::w(i) * Sb[c];
      a.G[(static_cast<size_t>(i) * 3 + c) * a.stride + gnode] = E::enc(v, fscale<S, ML>(i));
    }
  }
  for (int i = 0; i < FL::q; ++i) {
    size_t fnode = cell;
    if (a.fpull)
      fnode = vnode(wrap(px - FL::c(i, 0), a.nx), wrap(py - FL::c(i, 1), a.ny), wrap(pz - FL::c(i, 2), a.nz), a.nx, a.ny);
    a.F[static_cast<size_t>(i) * a.stride + fnode] = E::enc(f[i], fscale<S, FL>(i));
  }
}

// ------------------------------------------------------------------ canonical copies
// Canonical order: q fluid arrays, then m x 3 magnetic arrays, each of n nodes. Full values add
// the rest state f_rest (by value) and W_i b0; deviation copies add nothing.
struct VRest {
  double f[27];
  double b0[3];
  int deviations;
};
template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(256) void variant_get(VView<S, FL, ML> v, VRest r, double* dst) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= v.n) return;
  int x, y, z;
  vxyz(cell, v.geo.nx, v.geo.ny, x, y, z);
  for (int i = 0; i < FL::q; ++i)
    dst[static_cast<size_t>(i) * v.n + cell] = (r.deviations ? 0.0 : r.f[i]) + v.f(i, x, y, z);
  for (int i = 0; i < ML::m; ++i)
    for (int c = 0; c < 3; ++c)
      dst[(FL::q + static_cast<size_t>(i) * 3 + c) * v.n + cell] =
          (r.deviations ? 0.0 : ML::w(i) * r.b0[c]) + v.g(i, c, x, y, z);
}

template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(256) void variant_gather(VView<S, FL, ML> v, VRest r, const int64_t* cells,
                                                      int64_t cnt, double* out) {
  constexpr int K = FL::q + 3 * ML::m;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const int64_t cell = cells[k];
  if (cell < 0 || static_cast<size_t>(cell) >= v.n) {
    for (int q = 0; q < K; ++q) out[k * K + q] = NAN;
    return;
  }
  int x, y, z;
  vxyz(static_cast<size_t>(cell), v.geo.nx, v.geo.ny, x, y, z);
  for (int i = 0; i < FL::q; ++i) out[k * K + i] = (r.deviations ? 0.0 : r.f[i]) + v.f(i, x, y, z);
  for (int i = 0; i < ML::m; ++i)
    for (int c = 0; c < 3; ++c)
      out[k * K + FL::q + i * 3 + c] = (r.deviations ? 0.0 : ML::w(i) * r.b0[c]) + v.g(i, c, x, y, z);
}

template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(256) void variant_set(S* F, S* G, SetGeom geo, size_t n, int fpull, int gpull,
                                                   VRest r, const double* src) {
  using E = Enc<S>;
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= n) return;
  int x, y, z;
  vxyz(cell, geo.nx, geo.ny, x, y, z);
  for (int i = 0; i < FL::q; ++i) {
    size_t node = cell;
    if (fpull) node = vnode(wrap(x - FL::c(i, 0), geo.nx), wrap(y - FL::c(i, 1), geo.ny), wrap(z - FL::c(i, 2), geo.nz), geo.nx, geo.ny);
    F[static_cast<size_t>(i) * geo.stride + node] =
        E::enc(src[static_cast<size_t>(i) * n + cell] - (r.deviations ? 0.0 : r.f[i]), fscale<S, FL>(i));
  }
  for (int i = 0; i < ML::m; ++i) {
    size_t node = cell;
    if (gpull) node = vnode(wrap(x - ML::xi(i, 0), geo.nx), wrap(y - ML::xi(i, 1), geo.ny), wrap(z - ML::xi(i, 2), geo.nz), geo.nx, geo.ny);
    for (int c = 0; c < 3; ++c) {
      const size_t k = static_cast<size_t>(i) * 3 + c;
      G[k * geo.stride + node] =
          E::enc(src[(FL::q + k) * n + cell] - (r.deviations ? 0.0 : ML::w(i) * r.b0[c]), fscale<S, ML>(i));
    }
  }
}

// ------------------------------------------------------------------ node fields and reductions
template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(256) void variant_moments(VAux<S, FL, ML> a, double* rho, double* u, double* B,
                                                       double* J, double* divb) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.v.n) return;
  int x, y, z;
  vxyz(cell, a.v.geo.nx, a.v.geo.ny, x, y, z);
  double r, U[3], Bf[3], b[3], Jf[3], d;
  bool fin;
  node_q(a, x, y, z, r, U, Bf, b, Jf, d, fin);
  const size_t n = a.v.n;
  if (rho) rho[cell] = r;
  if (divb) divb[cell] = d;
  for (int c = 0; c < 3; ++c) {
    if (u) u[c * n + cell] = U[c];
    if (B) B[c * n + cell] = Bf[c];
    if (J) J[c * n + cell] = Jf[c];
  }
}

// One field component of u (field 0) or B (field 1) per node, for the spectra.
template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(256) void variant_component(VAux<S, FL, ML> a, int field, int comp, double* out) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.v.n) return;
  int x, y, z;
  vxyz(cell, a.v.geo.nx, a.v.geo.ny, x, y, z);
  double r, U[3], Bf[3], b[3], Jf[3], d;
  bool fin;
  node_q(a, x, y, z, r, U, Bf, b, Jf, d, fin);
  // selected without a runtime index into the arrays (which would put them in per-thread private memory)
  const double uc = comp == 0 ? U[0] : comp == 1 ? U[1] : U[2];
  const double bc = comp == 0 ? Bf[0] : comp == 1 ? Bf[1] : Bf[2];
  out[cell] = field == 0 ? uc : bc;
}

// Block partials of the FP64 reductions in the slot order of flame_reduce (fixed grid, fixed
// tree order).
constexpr int kVRedThreads = 256;
template <typename S, typename FL, typename ML>
__global__ __launch_bounds__(kVRedThreads) void variant_reduce(VAux<S, FL, ML> a, double* partials) {
  double acc[FLAME_NRED];
  for (int k = 0; k < FLAME_NRED; ++k) acc[k] = 0.0;
  const size_t step = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; cell < a.v.n; cell += step) {
    int x, y, z;
    vxyz(cell, a.v.geo.nx, a.v.geo.ny, x, y, z);
    double r, U[3], Bf[3], b[3], J[3], d;
    bool fin;
    node_q(a, x, y, z, r, U, Bf, b, J, d, fin);
    const double u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    acc[0] += 0.5 * u2;
    acc[1] += 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    acc[2] += U[0] * b[0] + U[1] * b[1] + U[2] * b[2];
    acc[3] += J[0] * J[0] + J[1] * J[1] + J[2] * J[2];
    acc[4] = fmax(acc[4], fabs(d));
    acc[5] += d * d;
    acc[6] = fmax(acc[6], sqrt(u2));
    acc[7] += (r - 1.0) * (r - 1.0);
    acc[8] += fin ? 0.0 : 1.0;
    acc[9] += r;
    for (int c = 0; c < 3; ++c) {
      acc[10 + c] += r * U[c];
      acc[13 + c] += Bf[c];
    }
  }
  __shared__ double sh[FLAME_NRED][kVRedThreads];
  for (int k = 0; k < FLAME_NRED; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (unsigned s = kVRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < FLAME_NRED; ++k) {
        const double o = sh[k][threadIdx.x + s];
        sh[k][threadIdx.x] = (k == 4 || k == 6) ? fmax(sh[k][threadIdx.x], o) : sh[k][threadIdx.x] + o;
      }
    __syncthreads();
  }
  if (threadIdx.x < FLAME_NRED) partials[blockIdx.x * FLAME_NRED + threadIdx.x] = sh[threadIdx.x][0];
}

// ------------------------------------------------------------------ host dispatch
template <typename S, typename FL, typename ML>
VAux<S, FL, ML> make_vaux(const flame_ctx* c) {
  using R = typename Enc<S>::R;
  const SetPtrs s = set_ptrs(c);
  VAux<S, FL, ML> a;
  a.v.F = static_cast<const S*>(s.f_src);
  a.v.G = static_cast<const S*>(s.g_src);
  a.v.fmode = s.fluid_aa ? (c->parity == 1 ? 1 : 0) : 2;
  a.v.gmode = s.mag_aa ? (c->parity == 1 ? 1 : 0) : 2;
  a.v.geo = SetGeom{c->p.nx, c->p.ny, c->p.nz, c->stride};
  a.v.n = c->n;
  a.force_u = static_cast<const R*>(c->p.force_u);
  a.force_b = static_cast<const R*>(c->p.force_b);
  for (int i = 0; i < 3; ++i) a.b0[i] = c->p.b0[i];
  a.alpha = c->p.d_i;
  a.omega_b = c->omega_b;
  a.emhd = c->p.magnetic == FLAME_MAGNETIC_EMHD;
  return a;
}

inline unsigned vblocks(size_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

// Calls fn(S{}, Fluid<Q>{}, Mag<M>{}) for the context's storage and lattices.
template <typename Fn>
hipError_t dispatch(const flame_params& p, Fn&& fn) {
  auto by_mag = [&](auto s, auto fl) -> hipError_t {
    switch (p.magnetic_lattice) {
      case FLAME_MAGNETIC_D3Q15: return fn(s, fl, Mag<15>{});
      case FLAME_MAGNETIC_D3Q27: return fn(s, fl, Mag<27>{});
      default: return fn(s, fl, Mag<7>{});
    }
  };
  auto by_fluid = [&](auto s) -> hipError_t {
    return p.fluid_lattice == FLAME_FLUID_D3Q19 ? by_mag(s, Fluid<19>{}) : by_mag(s, Fluid<27>{});
  };
  switch (p.storage) {
    case FLAME_F64: return by_fluid(double{});
    case FLAME_F32: return by_fluid(float{});
    default: return by_fluid(_Float16{});
  }
}

}  // namespace lattice

using namespace lattice;

hipError_t variant_launch_step(const flame_ctx* c, const SetPtrs& s) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    using R = typename Enc<S>::R;
    VStepArgs<S> a;
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
    a.stride = c->stride;
    a.k.omega = R(c->omega);
    a.k.omega_b = R(c->omega_b);
    a.k.alpha = R(c->p.d_i);
    for (int i = 0; i < 3; ++i) a.k.b0[i] = R(c->p.b0[i]);
    const unsigned tx = row_threads(c);
    const dim3 grid(((c->p.nx + tx - 1) / tx) * c->p.ny * c->p.nz);
    const bool bgk = c->p.collision == FLAME_COLLISION_BGK, emhd = c->p.magnetic == FLAME_MAGNETIC_EMHD;
    auto go = [&](auto aa, auto par) {
      constexpr bool AA = decltype(aa)::value;
      constexpr int PAR = decltype(par)::value;
      if (bgk && emhd) hipLaunchKernelGGL((variant_step<S, FL, ML, AA, PAR, true, true>), grid, dim3(tx), 0, c->stream, a);
      else if (bgk) hipLaunchKernelGGL((variant_step<S, FL, ML, AA, PAR, true, false>), grid, dim3(tx), 0, c->stream, a);
      else if (emhd) hipLaunchKernelGGL((variant_step<S, FL, ML, AA, PAR, false, true>), grid, dim3(tx), 0, c->stream, a);
      else hipLaunchKernelGGL((variant_step<S, FL, ML, AA, PAR, false, false>), grid, dim3(tx), 0, c->stream, a);
    };
    if (!s.fluid_aa) go(std::false_type{}, std::integral_constant<int, 0>{});
    else if (c->parity == 0) go(std::true_type{}, std::integral_constant<int, 0>{});
    else go(std::true_type{}, std::integral_constant<int, 1>{});
    return hipGetLastError();
  });
}

hipError_t variant_launch_init(const flame_ctx* c, const double* u, const double* b, const double* grad_u,
                               const double* grad_b) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    using R = typename Enc<S>::R;
    const SetPtrs s = set_ptrs(c);
    VInitArgs<S> a;
    a.F = static_cast<S*>(s.f_src);
    a.G = static_cast<S*>(s.g_src);
    a.u = u;
    a.b = b;
    a.gu = grad_u;
    a.gb = grad_b;
    a.force_u = static_cast<const R*>(c->p.force_u);
    a.force_b = static_cast<const R*>(c->p.force_b);
    for (int i = 0; i < 3; ++i) a.b0[i] = c->p.b0[i];
    a.omega = c->omega;
    a.omega_b = c->omega_b;
    a.alpha = c->p.d_i;
    a.noneq = c->p.init_noneq;
    a.emhd = c->p.magnetic == FLAME_MAGNETIC_EMHD;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.n = c->n;
    a.stride = c->stride;
    a.fpull = !s.fluid_aa;
    a.gpull = !s.mag_aa;
    hipLaunchKernelGGL((variant_init<S, FL, ML>), dim3(vblocks(c->n, 256)), dim3(256), 0, c->stream, a);
    return hipGetLastError();
  });
}

namespace {
VRest make_vrest(const flame_ctx* c, int deviations) {
  VRest r;
  for (int i = 0; i < 27; ++i) r.f[i] = c->frest[i];
  for (int i = 0; i < 3; ++i) r.b0[i] = c->p.b0[i];
  r.deviations = deviations;
  return r;
}
}  // namespace

hipError_t variant_launch_get(const flame_ctx* c, int deviations, double* dst) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    hipLaunchKernelGGL((variant_get<S, FL, ML>), dim3(vblocks(c->n, 256)), dim3(256), 0, c->stream,
                       make_vaux<S, FL, ML>(c).v, make_vrest(c, deviations), dst);
    return hipGetLastError();
  });
}

hipError_t variant_launch_gather(const flame_ctx* c, int deviations, const int64_t* cells, int64_t cnt, double* out) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    hipLaunchKernelGGL((variant_gather<S, FL, ML>), dim3(vblocks(static_cast<size_t>(cnt), 256)), dim3(256), 0,
                       c->stream, make_vaux<S, FL, ML>(c).v, make_vrest(c, deviations), cells, cnt, out);
    return hipGetLastError();
  });
}

hipError_t variant_launch_set(const flame_ctx* c, int deviations, const double* src) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    const SetPtrs s = set_ptrs(c);
    const SetGeom geo{c->p.nx, c->p.ny, c->p.nz, c->stride};
    hipLaunchKernelGGL((variant_set<S, FL, ML>), dim3(vblocks(c->n, 256)), dim3(256), 0, c->stream,
                       static_cast<S*>(s.f_src), static_cast<S*>(s.g_src), geo, c->n, s.fluid_aa ? 0 : 1,
                       s.mag_aa ? 0 : 1, make_vrest(c, deviations), src);
    return hipGetLastError();
  });
}

hipError_t variant_launch_moments(const flame_ctx* c, double* rho, double* u, double* b, double* j, double* divb) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    hipLaunchKernelGGL((variant_moments<S, FL, ML>), dim3(vblocks(c->n, 256)), dim3(256), 0, c->stream,
                       make_vaux<S, FL, ML>(c), rho, u, b, j, divb);
    return hipGetLastError();
  });
}

hipError_t variant_launch_component(const flame_ctx* c, int field, int comp, double* out) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    hipLaunchKernelGGL((variant_component<S, FL, ML>), dim3(vblocks(c->n, 256)), dim3(256), 0, c->stream,
                       make_vaux<S, FL, ML>(c), field, comp, out);
    return hipGetLastError();
  });
}

hipError_t variant_launch_reduce(const flame_ctx* c, double* partials) {
  return dispatch(c->p, [&](auto stag, auto fltag, auto mltag) -> hipError_t {
    using S = decltype(stag);
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    hipLaunchKernelGGL((variant_reduce<S, FL, ML>), dim3(c->red_blocks), dim3(kVRedThreads), 0, c->stream,
                       make_vaux<S, FL, ML>(c), partials);
    return hipGetLastError();
  });
}

void variant_rest(const flame_params& p, double* f_rest, double* g_rest) {
  auto fill = [&](auto fltag, auto mltag) {
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    const double* B0 = p.b0;
    const double b2 = B0[0] * B0[0] + B0[1] * B0[1] + B0[2] * B0[2];
    if (f_rest)
      for (int i = 0; i < FL::q; ++i) {
        const double cb = FL::c(i, 0) * B0[0] + FL::c(i, 1) * B0[1] + FL::c(i, 2) * B0[2];
        f_rest[i] = FL::w(i) + FL::w(i) * 4.5 * (0.5 * b2 * (FL::speed2(i) - 1.0 / 3.0) - cb * cb);
      }
    if (g_rest)
      for (int i = 0; i < ML::m; ++i)
        for (int c = 0; c < 3; ++c) g_rest[i * 3 + c] = ML::w(i) * B0[c];
  };
  auto by_mag = [&](auto fl) {
    switch (p.magnetic_lattice) {
      case FLAME_MAGNETIC_D3Q15: fill(fl, Mag<15>{}); break;
      case FLAME_MAGNETIC_D3Q27: fill(fl, Mag<27>{}); break;
      default: fill(fl, Mag<7>{}); break;
    }
  };
  if (p.fluid_lattice == FLAME_FLUID_D3Q19) by_mag(Fluid<19>{});
  else by_mag(Fluid<27>{});
}

}  // namespace flame
