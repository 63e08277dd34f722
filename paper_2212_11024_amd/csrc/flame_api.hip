// C ABI of the library (include/flame.h): validation, buffer bookkeeping, the initial
// state, canonical access, node fields, FP64 reductions and shell spectra.

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "flame_internal.h"

namespace flame {

// Rest populations f^mhd(0)(1, 0, b0), passed to kernels by value.
struct Rest {
  double f[27];
  double b0[3];
};

// ------------------------------------------------------------------ canonical view
// Read access to the current state in canonical order, for the auxiliary kernels. Returns
// decoded deviations as double.
template <typename S>
struct View {
  const S* F;
  const S* G;
  // addressing of the canonical population i at node x:
  //   0: slot i at x (AA even step); 1: slot opp(i) at x - c_i (AA odd step);
  //   2: slot i at x - c_i (two-lattice pull: the source copy holds post-collision values)
  int fmode;
  int gmode;
  int nx, ny, nz;
  size_t n;
  size_t stride;   // elements between population arrays

  // node index in 32-bit arithmetic: flame_init refuses grids of 2^32 nodes or more
  __device__ size_t node(int x, int y, int z) const {
    return (static_cast<size_t>(z) * ny + y) * nx + x;
  }
  // element of F / G holding canonical population i (component c) of node (x, y, z), for the
  // trace export
  __device__ size_t fidx(int i, int x, int y, int z) const {
    return fmode == 0 ? static_cast<size_t>(i) * stride + node(x, y, z)
                      : static_cast<size_t>(fmode == 1 ? oppq(i) : i) * stride +
                            node(wrap(x - cq(i, 0), nx), wrap(y - cq(i, 1), ny), wrap(z - cq(i, 2), nz));
  }
  __device__ size_t gidx(int i, int c, int x, int y, int z) const {
    return gmode == 0 ? static_cast<size_t>(i * 3 + c) * stride + node(x, y, z)
                      : static_cast<size_t>((gmode == 1 ? oppm(i) : i) * 3 + c) * stride +
                            node(wrap(x - xim(i, 0), nx), wrap(y - xim(i, 1), ny), wrap(z - xim(i, 2), nz));
  }
  // the same with the addressing mode fixed at compile time (no branch per access, so that a
  // node's loads can all be in flight together)
  template <int M>
  __device__ double fm(int i, int x, int y, int z) const {
    const size_t idx = M == 0 ? static_cast<size_t>(i) * stride + node(x, y, z)
                              : static_cast<size_t>(M == 1 ? oppq(i) : i) * stride +
                                    node(wrap(x - cq(i, 0), nx), wrap(y - cq(i, 1), ny), wrap(z - cq(i, 2), nz));
    return static_cast<double>(F[idx]) / Enc<S>::fscale(i);
  }
  template <int M>
  __device__ double gm(int i, int c, int x, int y, int z) const {
    const size_t idx = M == 0 ? static_cast<size_t>(i * 3 + c) * stride + node(x, y, z)
                              : static_cast<size_t>((M == 1 ? oppm(i) : i) * 3 + c) * stride +
                                    node(wrap(x - xim(i, 0), nx), wrap(y - xim(i, 1), ny), wrap(z - xim(i, 2), nz));
    return static_cast<double>(G[idx]) / Enc<S>::mscale(i);
  }
  // runtime mode: the element index is selected, then one load
  __device__ double f(int i, int x, int y, int z) const {
    size_t idx = fmode == 0 ? static_cast<size_t>(i) * stride + node(x, y, z)
                            : static_cast<size_t>(fmode == 1 ? oppq(i) : i) * stride +
                                  node(wrap(x - cq(i, 0), nx), wrap(y - cq(i, 1), ny), wrap(z - cq(i, 2), nz));
    return static_cast<double>(F[idx]) / Enc<S>::fscale(i);
  }
  __device__ double g(int i, int c, int x, int y, int z) const {
    size_t idx = gmode == 0 ? static_cast<size_t>(i * 3 + c) * stride + node(x, y, z)
                            : static_cast<size_t>((gmode == 1 ? oppm(i) : i) * 3 + c) * stride +
                                  node(wrap(x - xim(i, 0), nx), wrap(y - xim(i, 1), ny), wrap(z - xim(i, 2), nz));
    return static_cast<double>(G[idx]) / Enc<S>::mscale(i);
  }
};

// All populations of node (x, y, z), decoded, in canonical order; the mode switch is taken once
// per node.
template <int M, typename S>
__device__ __forceinline__ void view_fluid(const View<S>& v, int x, int y, int z, double (&f)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) f[i] = v.template fm<M>(i, x, y, z);
}
template <int M, typename S>
__device__ __forceinline__ void view_magnetic(const View<S>& v, int x, int y, int z, double (&g)[kM]) {
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) g[i * 3 + c] = v.template gm<M>(i, c, x, y, z);
}
template <typename S>
__device__ __forceinline__ void view_node(const View<S>& v, int x, int y, int z, double (&f)[kQ], double (&g)[kM]) {
  if (v.fmode == 0) view_fluid<0>(v, x, y, z, f);
  else if (v.fmode == 1) view_fluid<1>(v, x, y, z, f);
  else view_fluid<2>(v, x, y, z, f);
  if (v.gmode == 0) view_magnetic<0>(v, x, y, z, g);
  else if (v.gmode == 1) view_magnetic<1>(v, x, y, z, g);
  else view_magnetic<2>(v, x, y, z, g);
}

// Where a writer of the canonical state (initial state, set) puts population i of node
// (x, y, z): its own slot for in-place sets; for pull sets the slot at x - c_i, which is where
// the next step at node x pulls population i from.
struct Placement {
  bool fpull, gpull;
  int nx, ny, nz;
  __device__ size_t f(int i, int x, int y, int z) const {
    if (fpull) { x = wrap(x - cq(i, 0), nx); y = wrap(y - cq(i, 1), ny); z = wrap(z - cq(i, 2), nz); }
    return (static_cast<size_t>(z) * ny + y) * nx + x;
  }
  __device__ size_t g(int i, int x, int y, int z) const {
    if (gpull) { x = wrap(x - xim(i, 0), nx); y = wrap(y - xim(i, 1), ny); z = wrap(z - xim(i, 2), nz); }
    return (static_cast<size_t>(z) * ny + y) * nx + x;
  }
};

// Node quantities in FP64 from the canonical view.
struct NodeQ {
  double rho, U[3], B[3], b[3], J[3], divb;
  bool finite;
};

template <typename S>
struct AuxArgs {
  View<S> v;
  const typename Enc<S>::R* force_u;
  const typename Enc<S>::R* force_b;
  double b0[3];
  double alpha, omega_b;
  int stencil;
  int emhd;     // electron MHD: J from the moments with the bulk velocity taken as zero
};

template <typename S>
__device__ double field_fluct(const AuxArgs<S>& a, int comp, int x, int y, int z) {
  double s = a.v.g(0, comp, x, y, z);
  for (int i = 1; i < 7; ++i) s += a.v.g(i, comp, x, y, z);
  if (a.force_b) s += 0.5 * static_cast<double>(a.force_b[static_cast<size_t>(comp) * a.v.n + a.v.node(x, y, z)]);
  return s;
}
// the same with the magnetic addressing mode fixed at compile time (same order of the sum)
template <int M, typename S>
__device__ __forceinline__ double field_fluct_m(const AuxArgs<S>& a, int comp, int x, int y, int z) {
  double s = a.v.template gm<M>(0, comp, x, y, z);
#pragma unroll
  for (int i = 1; i < 7; ++i) s += a.v.template gm<M>(i, comp, x, y, z);
  if (a.force_b) s += 0.5 * static_cast<double>(a.force_b[static_cast<size_t>(comp) * a.v.n + a.v.node(x, y, z)]);
  return s;
}
// J = central-difference curl of b at node (x, y, z)
template <int M, typename S>
__device__ __forceinline__ void curl_b(const AuxArgs<S>& a, int x, int y, int z, double (&J)[3]) {
  const View<S>& v = a.v;
  const int xp = wrap(x + 1, v.nx), xm = wrap(x - 1, v.nx);
  const int yp = wrap(y + 1, v.ny), ym = wrap(y - 1, v.ny);
  const int zp = wrap(z + 1, v.nz), zm = wrap(z - 1, v.nz);
  J[0] = 0.5 * (field_fluct_m<M>(a, 2, x, yp, z) - field_fluct_m<M>(a, 2, x, ym, z))
       - 0.5 * (field_fluct_m<M>(a, 1, x, y, zp) - field_fluct_m<M>(a, 1, x, y, zm));
  J[1] = 0.5 * (field_fluct_m<M>(a, 0, x, y, zp) - field_fluct_m<M>(a, 0, x, y, zm))
       - 0.5 * (field_fluct_m<M>(a, 2, xp, y, z) - field_fluct_m<M>(a, 2, xm, y, z));
  J[2] = 0.5 * (field_fluct_m<M>(a, 1, xp, y, z) - field_fluct_m<M>(a, 1, xm, y, z))
       - 0.5 * (field_fluct_m<M>(a, 0, x, yp, z) - field_fluct_m<M>(a, 0, x, ym, z));
}

template <typename S>
__device__ NodeQ node_quantities(const AuxArgs<S>& a, int x, int y, int z) {
  NodeQ q;
  const View<S>& v = a.v;
  const size_t cell = v.node(x, y, z);
  // unrolled, so that f and g stay in registers (a runtime index would put them in per-thread private memory)
  double f[kQ], g[kM];
  view_node(v, x, y, z, f, g);
  bool fin = true;
#pragma unroll
  for (int i = 0; i < kQ; ++i) fin = fin && isfinite(f[i]);
#pragma unroll
  for (int k = 0; k < kM; ++k) fin = fin && isfinite(g[k]);
  q.finite = fin;
  double drho = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += f[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) j[c] += cq(i, c) * f[i];
  }
  q.rho = 1.0 + drho;
  for (int c = 0; c < 3; ++c) {
    const double F = a.force_u ? static_cast<double>(a.force_u[static_cast<size_t>(c) * v.n + cell]) : 0.0;
    q.U[c] = (j[c] + 0.5 * F) / q.rho;
  }
  double lam[3][3];
  double bb[3];
  magnetic_moments(g, bb, lam);
  for (int c = 0; c < 3; ++c) {
    const double src = a.force_b ? static_cast<double>(a.force_b[static_cast<size_t>(c) * v.n + cell]) : 0.0;
    q.b[c] = bb[c] + 0.5 * src;
    q.B[c] = a.b0[c] + q.b[c];
  }
  if (!a.stencil) {
    const double zero[3] = {0.0, 0.0, 0.0};
    current_from_moments(lam, a.emhd ? zero : q.U, q.B, a.alpha, a.omega_b, q.J);
  } else if (v.gmode == 0) {
    curl_b<0>(a, x, y, z, q.J);
  } else if (v.gmode == 1) {
    curl_b<1>(a, x, y, z, q.J);
  } else {
    curl_b<2>(a, x, y, z, q.J);
  }
  q.divb = -4.0 * a.omega_b * (lam[0][0] + lam[1][1] + lam[2][2]);
  return q;
}

// cell < 2^32 (flame_init refuses larger grids), so 32-bit division suffices
__device__ __forceinline__ void node_xyz(size_t cell, int nx, int ny, int& x, int& y, int& z) {
  x = static_cast<int>(cell % nx);
  const size_t r = cell / nx;
  y = static_cast<int>(r % ny);
  z = static_cast<int>(r / ny);
}

// ------------------------------------------------------------------ initial state
template <typename S>
struct InitArgs {
  using R = typename Enc<S>::R;
  S* F;
  S* G;
  const double* u;
  const double* b;
  const double* gu;   // [3][3][n] or null
  const double* gb;
  const R* force_u;
  const R* force_b;
  double b0[3];
  double omega, omega_b, alpha;
  int noneq;
  int emhd;
  int nx, ny, nz;
  size_t n;
  size_t stride;
  Placement at;
};

template <typename S>
__global__ __launch_bounds__(256) void init_kernel(InitArgs<S> a) {
  using E = Enc<S>;
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.n) return;
  const size_t n = a.n;
  int px, py, pz;
  node_xyz(cell, a.nx, a.ny, px, py, pz);
  double U[3], b[3], B[3], F[3] = {0, 0, 0}, Sb[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) {
    U[c] = a.u[c * n + cell];
    b[c] = a.b[c * n + cell];
    B[c] = a.b0[c] + b[c];
    if (a.force_u) F[c] = static_cast<double>(a.force_u[c * n + cell]);
    if (a.force_b) Sb[c] = static_cast<double>(a.force_b[c * n + cell]);
  }
  // gradients: given, or (with the non-equilibrium initialisation) central differences on the grid
  auto central = [&](const double* v, double (&g)[3][3]) {
    auto at = [&](int x, int y, int z) { return (static_cast<size_t>(z) * a.ny + y) * a.nx + x; };
    const size_t xm = at(wrap(px - 1, a.nx), py, pz), xp = at(wrap(px + 1, a.nx), py, pz);
    const size_t ym = at(px, wrap(py - 1, a.ny), pz), yp = at(px, wrap(py + 1, a.ny), pz);
    const size_t zm = at(px, py, wrap(pz - 1, a.nz)), zp = at(px, py, wrap(pz + 1, a.nz));
    for (int c = 0; c < 3; ++c) {
      const double* vc = v + c * n;
      g[0][c] = 0.5 * (vc[xp] - vc[xm]);
      g[1][c] = 0.5 * (vc[yp] - vc[ym]);
      g[2][c] = 0.5 * (vc[zp] - vc[zm]);
    }
  };
  double gu[3][3] = {}, gb[3][3] = {};
  bool have_gu = a.gu != nullptr, have_gb = a.gb != nullptr;
  if (a.gu) {
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) gu[p][q] = a.gu[(p * 3 + q) * n + cell];
  } else if (a.noneq) {
    central(a.u, gu);
    have_gu = true;
  }
  if (a.gb) {
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) gb[p][q] = a.gb[(p * 3 + q) * n + cell];
  } else if (a.noneq) {
    central(a.b, gb);
    have_gb = true;
  }
  PhysConst<double> k;
  k.omega = a.omega;
  k.omega_b = a.omega_b;
  k.alpha = a.alpha;
  for (int c = 0; c < 3; ++c) k.b0[c] = a.b0[c];
  InitFlags fl;
  fl.fluid_noneq = a.noneq && have_gu;
  fl.mag_noneq = a.noneq && have_gb;
  fl.has_H = have_gb;
  fl.emhd = a.emhd != 0;
  double f[kQ], g[kM];
  init_node(U, b, gu, gb, F, Sb, k, fl, f, g);
  for (int i = 0; i < kQ; ++i)
    a.F[static_cast<size_t>(i) * a.stride + a.at.f(i, px, py, pz)] = E::enc(f[i], E::fscale(i));
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c)
      a.G[static_cast<size_t>(i * 3 + c) * a.stride + a.at.g(i, px, py, pz)] = E::enc(g[i * 3 + c], E::mscale(i));
}

// ------------------------------------------------------------------ canonical copies
template <typename S>
__global__ __launch_bounds__(256) void get_kernel(View<S> v, Rest r, double* dst) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= v.n) return;
  int x, y, z;
  node_xyz(cell, v.nx, v.ny, x, y, z);
  for (int i = 0; i < kQ; ++i) dst[static_cast<size_t>(i) * v.n + cell] = r.f[i] + v.f(i, x, y, z);
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c)
      dst[(27 + static_cast<size_t>(i * 3 + c)) * v.n + cell] = wm(i) * r.b0[c] + v.g(i, c, x, y, z);
}

template <typename S>
__global__ __launch_bounds__(256) void set_kernel(S* F, S* G, size_t n, size_t stride, Placement at, Rest r,
                                                  const double* src) {
  using E = Enc<S>;
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= n) return;
  int x, y, z;
  node_xyz(cell, at.nx, at.ny, x, y, z);
  for (int i = 0; i < kQ; ++i)
    F[static_cast<size_t>(i) * stride + at.f(i, x, y, z)] =
        E::enc(src[static_cast<size_t>(i) * n + cell] - r.f[i], E::fscale(i));
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c) {
      const size_t k = static_cast<size_t>(i * 3 + c);
      G[k * stride + at.g(i, x, y, z)] = E::enc(src[(27 + k) * n + cell] - wm(i) * r.b0[c], E::mscale(i));
    }
}

// Trace lattice of the current state (two-lattice pull layout, node stride n): canonical
// population i of node x goes to slot i at x - c_i, where a pull step at x reads it. The stored
// values are moved without decoding, so the copy is exact.
template <typename S>
__global__ __launch_bounds__(256) void export_kernel(View<S> v, S* lat) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= v.n) return;
  int x, y, z;
  node_xyz(cell, v.nx, v.ny, x, y, z);
  for (int i = 0; i < kQ; ++i)
    lat[static_cast<size_t>(i) * v.n + v.node(wrap(x - cq(i, 0), v.nx), wrap(y - cq(i, 1), v.ny),
                                              wrap(z - cq(i, 2), v.nz))] = v.F[v.fidx(i, x, y, z)];
  for (int i = 0; i < 7; ++i) {
    const size_t dn = v.node(wrap(x - xim(i, 0), v.nx), wrap(y - xim(i, 1), v.ny), wrap(z - xim(i, 2), v.nz));
    for (int c = 0; c < 3; ++c) lat[static_cast<size_t>(kQ + i * 3 + c) * v.n + dn] = v.G[v.gidx(i, c, x, y, z)];
  }
}

template <typename S>
__global__ __launch_bounds__(256) void gather_kernel(View<S> v, Rest r, const int64_t* cells, int64_t cnt,
                                                     double* out) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const int64_t cell = cells[k];
  if (cell < 0 || static_cast<size_t>(cell) >= v.n) {
    for (int q = 0; q < 48; ++q) out[k * 48 + q] = NAN;
    return;
  }
  int x, y, z;
  node_xyz(static_cast<size_t>(cell), v.nx, v.ny, x, y, z);
  for (int i = 0; i < kQ; ++i) out[k * 48 + i] = r.f[i] + v.f(i, x, y, z);
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c) out[k * 48 + 27 + i * 3 + c] = wm(i) * r.b0[c] + v.g(i, c, x, y, z);
}

// ------------------------------------------------------------------ node fields
template <typename S>
__global__ __launch_bounds__(256) void moments_kernel(AuxArgs<S> a, double* rho, double* u, double* B,
                                                      double* J, double* divb) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.v.n) return;
  int x, y, z;
  node_xyz(cell, a.v.nx, a.v.ny, x, y, z);
  const NodeQ q = node_quantities(a, x, y, z);
  const size_t n = a.v.n;
  if (rho) rho[cell] = q.rho;
  if (divb) divb[cell] = q.divb;
  for (int c = 0; c < 3; ++c) {
    if (u) u[c * n + cell] = q.U[c];
    if (B) B[c * n + cell] = q.B[c];
    if (J) J[c * n + cell] = q.J[c];
  }
}

// ------------------------------------------------------------------ adjoint of the node fields
// lam = d loss / d(canonical deviations) for a loss of the node fields u = (j + F/2) / rho and
// B = b0 + sum g + S/2: du_a / df_i = (c_ia - u_a) / rho, dB_c / dg_{i,c} = 1.
template <typename S>
__global__ __launch_bounds__(256) void adjoint_fields_kernel(View<S> v, const typename Enc<S>::R* force_u,
                                                             const double* dl_du, const double* dl_db,
                                                             typename Enc<S>::R* lam) {
  using R = typename Enc<S>::R;
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= v.n) return;
  const size_t n = v.n;
  int x, y, z;
  node_xyz(cell, v.nx, v.ny, x, y, z);
  double lu[3] = {0, 0, 0}, U[3] = {0, 0, 0}, rho = 1.0;
  if (dl_du) {
    double j[3] = {0, 0, 0};
    for (int i = 0; i < kQ; ++i) {
      const double fi = v.f(i, x, y, z);
      rho += fi;
      for (int c = 0; c < 3; ++c) j[c] += cq(i, c) * fi;
    }
    for (int c = 0; c < 3; ++c) {
      const double F = force_u ? static_cast<double>(force_u[c * n + cell]) : 0.0;
      U[c] = (j[c] + 0.5 * F) / rho;
      lu[c] = dl_du[c * n + cell];
    }
  }
  for (int i = 0; i < kQ; ++i) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) s += lu[c] * (cq(i, c) - U[c]);
    lam[static_cast<size_t>(i) * n + cell] = static_cast<R>(s / rho);
  }
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c)
      lam[static_cast<size_t>(kQ + i * 3 + c) * n + cell] = static_cast<R>(dl_db ? dl_db[c * n + cell] : 0.0);
}

// ------------------------------------------------------------------ reductions
constexpr int kRedThreads = 256;
constexpr int kRedBlocksMax = 2048;

// Per-block partials: sums in every slot except 4 and 6 (maxima). Fixed grid and a fixed
// tree order make the result bitwise reproducible. Two blocks per CU at least: without that
// bound the FP64 instantiation takes 261 VGPRs (one wave per SIMD) and runs slower than with
// the few spills the bound costs.
template <typename S>
__global__ __launch_bounds__(kRedThreads, 2) void reduce_kernel(AuxArgs<S> a, double* partials) {
  double acc[FLAME_NRED];
  for (int k = 0; k < FLAME_NRED; ++k) acc[k] = 0.0;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; cell < a.v.n; cell += stride) {
    int x, y, z;
    node_xyz(cell, a.v.nx, a.v.ny, x, y, z);
    const NodeQ q = node_quantities(a, x, y, z);
    const double u2 = q.U[0] * q.U[0] + q.U[1] * q.U[1] + q.U[2] * q.U[2];
    acc[0] += 0.5 * u2;
    acc[1] += 0.5 * (q.b[0] * q.b[0] + q.b[1] * q.b[1] + q.b[2] * q.b[2]);
    acc[2] += q.U[0] * q.b[0] + q.U[1] * q.b[1] + q.U[2] * q.b[2];
    acc[3] += q.J[0] * q.J[0] + q.J[1] * q.J[1] + q.J[2] * q.J[2];
    acc[4] = fmax(acc[4], fabs(q.divb));
    acc[5] += q.divb * q.divb;
    acc[6] = fmax(acc[6], sqrt(u2));
    acc[7] += (q.rho - 1.0) * (q.rho - 1.0);
    acc[8] += q.finite ? 0.0 : 1.0;
    acc[9] += q.rho;
    for (int c = 0; c < 3; ++c) {
      acc[10 + c] += q.rho * q.U[c];
      acc[13 + c] += q.B[c];
    }
  }
  __shared__ double sh[FLAME_NRED][kRedThreads];
  for (int k = 0; k < FLAME_NRED; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (unsigned s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int k = 0; k < FLAME_NRED; ++k) {
        const double o = sh[k][threadIdx.x + s];
        sh[k][threadIdx.x] = (k == 4 || k == 6) ? fmax(sh[k][threadIdx.x], o) : sh[k][threadIdx.x] + o;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < FLAME_NRED) partials[blockIdx.x * FLAME_NRED + threadIdx.x] = sh[threadIdx.x][0];
}

// Fixed-order merge of the block partials of reduce_kernel into the FLAME_NRED results: thread k
// runs over the blocks in order for slot k (sums; maxima for slots 4 and 6) and normalises the
// slot as flame_reduce documents (node averages, rms, plain sums and maxima).
__global__ __launch_bounds__(64) void reduce_merge_kernel(const double* partials, int blocks, double n,
                                                          double* out) {
  const int k = threadIdx.x;
  if (k >= FLAME_NRED) return;
  double acc = 0.0;
  for (int b = 0; b < blocks; ++b) {
    const double v = partials[static_cast<size_t>(b) * FLAME_NRED + k];
    acc = (k == 4 || k == 6) ? fmax(acc, v) : acc + v;
  }
  if (k <= 3) acc = acc / n;
  else if (k == 5 || k == 7) acc = sqrt(acc / n);
  out[k] = acc;
}

}  // namespace flame

// Block partials of the allocation-free reductions (flame_reduce_noalloc): one row of FLAME_NRED
// doubles per reduction block, kRedBlocksMax rows (256 KiB). Each GPU the library runs on holds its
// own copy until the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (see scratch_address), never by this name.
static __device__ __align__(256) double scratch[flame::kRedBlocksMax * FLAME_NRED];

namespace flame {

// ------------------------------------------------------------------ spectra
template <typename S>
__global__ __launch_bounds__(256) void field_component_kernel(AuxArgs<S> a, int field, int comp, double* out) {
  const size_t cell = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= a.v.n) return;
  int x, y, z;
  node_xyz(cell, a.v.nx, a.v.ny, x, y, z);
  const View<S>& v = a.v;
  if (field == 0) {
    double drho = 0, j = 0;
    for (int i = 0; i < kQ; ++i) {
      const double fi = v.f(i, x, y, z);
      drho += fi;
      j += cq(i, comp) * fi;
    }
    const double F = a.force_u ? static_cast<double>(a.force_u[comp * v.n + cell]) : 0.0;
    out[cell] = (j + 0.5 * F) / (1.0 + drho);
  } else {
    out[cell] = a.b0[comp] + field_fluct(a, comp, x, y, z);
  }
}

constexpr int kSpecShellsMax = 4096;

__device__ __forceinline__ int signed_freq(int idx, int n) { return idx <= (n - 1) / 2 ? idx : idx - n; }

// Shell binning without atomics. A binning block is one wavefront; it visits its entries in the
// fixed order of a grid-stride loop, 64 at a time, and adds each group's contributions shell by
// shell: the lanes holding one shell are summed by a fixed tree across the wavefront (the other
// lanes contribute +0), and lane 0 adds that sum to the block's LDS bins, which only it writes.
// The block partials are then merged in block order (bin_merge_kernel). Every sum therefore has
// one fixed order for a given grid, and spectra are bitwise reproducible.
constexpr int kBinThreads = 64;
constexpr int kBinBlocksMax = 2048;

// Lane 0 receives the sum of x over the 64 lanes, in a fixed tree order.
__device__ __forceinline__ double wave_sum_fixed(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, kBinThreads);
  return x;
}

// Add v to bins[shell] for every lane (shell < 0: nothing). Called by all 64 lanes together.
__device__ __forceinline__ void bin_group(double* bins, int shell, double v) {
  unsigned long long pending = __ballot(shell >= 0);
  while (pending) {
    const int leader = __ffsll(static_cast<long long>(pending)) - 1;
    const int s = __shfl(shell, leader, kBinThreads);
    const bool mine = shell == s;
    const double sum = wave_sum_fixed(mine ? v : 0.0);
    if (threadIdx.x == 0) bins[s] += sum;
    pending &= ~__ballot(mine);
  }
}

// Half-spectrum (nz, ny, nx/2+1) of an r2c transform; each entry stands for itself and, for
// 0 < kx < nx - kx, its conjugate mirror at -k (same shell). Each entry adds w |X|^2 norm2 to
// its shell: w = 1/2 for the energy spectrum; w = |q|^2, q_a = 2 pi k_a / n_a, for the
// dissipation spectrum (k2 set). Block partials [gridDim.x][nshells].
__global__ __launch_bounds__(kBinThreads) void shell_bin_kernel(const hipfftDoubleComplex* X, int nx, int ny,
                                                                int nz, int nshells, double norm2, int k2,
                                                                double* partials) {
  extern __shared__ double bins[];
  for (int s = threadIdx.x; s < nshells; s += blockDim.x) bins[s] = 0.0;
  __syncthreads();
  const int nxh = nx / 2 + 1;
  const size_t total = static_cast<size_t>(nz) * ny * nxh;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  // the loop bound is uniform over the wavefront, so every lane takes part in every group
  for (size_t base = static_cast<size_t>(blockIdx.x) * blockDim.x; base < total; base += stride) {
    const size_t k = base + threadIdx.x;
    int shell = -1;
    double v = 0.0;
    if (k < total) {
      const int kx = static_cast<int>(k % nxh);
      const size_t r = k / nxh;
      const int ky = static_cast<int>(r % ny);
      const int kz = static_cast<int>(r / ny);
      const double fx = kx, fy = signed_freq(ky, ny), fz = signed_freq(kz, nz);
      shell = static_cast<int>(floor(sqrt(fx * fx + fy * fy + fz * fz) + 0.5));
      if (shell < nshells) {
        const double re = X[k].x, im = X[k].y;
        const double mult = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
        double w = 0.5;
        if (k2) {
          const double qx = (2.0 * M_PI / nx) * fx, qy = (2.0 * M_PI / ny) * fy, qz = (2.0 * M_PI / nz) * fz;
          w = qx * qx + qy * qy + qz * qz;
        }
        v = mult * w * (re * re + im * im) * norm2;
      } else {
        shell = -1;
      }
    }
    bin_group(bins, shell, v);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nshells; s += blockDim.x) partials[static_cast<size_t>(blockIdx.x) * nshells + s] = bins[s];
}

// out[t][s] = sum over blocks, in block order, of partials[t][block][s] (terms t < gridDim.y).
__global__ __launch_bounds__(256) void bin_merge_kernel(const double* partials, int blocks, int nshells,
                                                        double* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshells) return;
  const size_t t = blockIdx.y;
  const double* p = partials + t * blocks * nshells + s;
  double acc = 0.0;
  for (int b = 0; b < blocks; ++b) acc += p[static_cast<size_t>(b) * nshells];
  out[t * nshells + s] = acc;
}

// ------------------------------------------------------------------ energy transfer
// Derivative wavenumber 2 pi k / n of the DFT index idx (signed), 0 on the Nyquist index of an
// even axis (that mode's derivative is not a real field).
__device__ __forceinline__ double deriv_q(int idx, int n) {
  return 2 * idx == n ? 0.0 : (2.0 * M_PI / n) * signed_freq(idx, n);
}

__device__ __forceinline__ void half_index(size_t k, int nx, int ny, int& kx, int& ky, int& kz) {
  const int nxh = nx / 2 + 1;
  kx = static_cast<int>(k % nxh);
  const size_t r = k / nxh;
  ky = static_cast<int>(r % ny);
  kz = static_cast<int>(r / ny);
}

// out = i q_axis X / ncell on the half spectrum: the inverse real transform of out is the
// derivative along axis of the field whose unnormalised forward transform is X.
__global__ __launch_bounds__(256) void spectral_derivative_kernel(const hipfftDoubleComplex* X, int nx, int ny,
                                                                  int nz, int axis, double inv_n,
                                                                  hipfftDoubleComplex* out) {
  const size_t total = static_cast<size_t>(nz) * ny * (nx / 2 + 1);
  const size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= total) return;
  int kx, ky, kz;
  half_index(k, nx, ny, kx, ky, kz);
  const double q = (axis == 0 ? deriv_q(kx, nx) : axis == 1 ? deriv_q(ky, ny) : deriv_q(kz, nz)) * inv_n;
  const hipfftDoubleComplex x = X[k];
  out[k] = make_hipDoubleComplex(-q * x.y, q * x.x);
}

// acc = (first ? 0 : acc) + a * b, node by node.
__global__ __launch_bounds__(256) void product_accumulate_kernel(double* acc, const double* a, const double* b,
                                                                 size_t n, int first) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  acc[i] = (first ? 0.0 : acc[i]) + a[i] * b[i];
}

// out = component comp of P x Q, with P and Q three consecutive arrays of n nodes.
__global__ __launch_bounds__(256) void cross_component_kernel(const double* P, const double* Q, int comp, size_t n,
                                                              double* out) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (comp + 1) % 3, d = (comp + 2) % 3;
  out[i] = P[c * n + i] * Q[d * n + i] - P[d * n + i] * Q[c * n + i];
}

// Per-block shell sums of one transfer summand over the half spectrum (entries with
// 0 < kx < nx - kx stand for their mirror too, whose summand is equal). kind 0:
// sign Re[conj(X) Y]; kind 1: -sign Re[i Y (conj(B_hat) x q)_comp] = -sign Re[conj(B_hat) . (i q x Y e_comp)]
// summed over comp by the caller, with B_hat the three transforms in Bh. Adds into partials
// unless first is set. Binned without atomics, as shell_bin_kernel.
__global__ __launch_bounds__(kBinThreads) void transfer_bin_kernel(int kind, const hipfftDoubleComplex* X,
                                                                   const hipfftDoubleComplex* Y,
                                                                   const hipfftDoubleComplex* Bh, int comp,
                                                                   double sign, int nx, int ny, int nz, int nshells,
                                                                   double norm2, int first, double* partials) {
  extern __shared__ double bins[];
  for (int s = threadIdx.x; s < nshells; s += blockDim.x) bins[s] = 0.0;
  __syncthreads();
  const size_t nh = static_cast<size_t>(nz) * ny * (nx / 2 + 1);
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t base = static_cast<size_t>(blockIdx.x) * blockDim.x; base < nh; base += stride) {
    const size_t k = base + threadIdx.x;
    int shell = -1;
    double v = 0.0;
    if (k < nh) {
      int kx, ky, kz;
      half_index(k, nx, ny, kx, ky, kz);
      const double fx = kx, fy = signed_freq(ky, ny), fz = signed_freq(kz, nz);
      shell = static_cast<int>(floor(sqrt(fx * fx + fy * fy + fz * fz) + 0.5));
      if (shell < nshells) {
        const hipfftDoubleComplex y = Y[k];
        if (kind == 0) {
          const hipfftDoubleComplex x = X[k];
          v = sign * (x.x * y.x + x.y * y.y);
        } else {
          const double q[3] = {deriv_q(kx, nx), deriv_q(ky, ny), deriv_q(kz, nz)};
          const int c = (comp + 1) % 3, d = (comp + 2) % 3;
          const size_t plane = nh;
          const hipfftDoubleComplex bc = Bh[c * plane + k], bd = Bh[d * plane + k];
          // z = (conj(B_hat) x q)_comp = conj(B_c) q_d - conj(B_d) q_c
          const double zr = bc.x * q[d] - bd.x * q[c];
          const double zi = -bc.y * q[d] + bd.y * q[c];
          // -Re[i y z] = Im[y z]
          v = sign * (y.x * zi + y.y * zr);
        }
        const double mult = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
        v = mult * v * norm2;
      } else {
        shell = -1;
      }
    }
    bin_group(bins, shell, v);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nshells; s += blockDim.x) {
    double& out = partials[static_cast<size_t>(blockIdx.x) * nshells + s];
    out = first ? bins[s] : out + bins[s];
  }
}

}  // namespace flame

using namespace flame;

// ====================================================================== host side
namespace {

thread_local std::string g_init_error;

flame_status fail(flame_ctx* c, flame_status code, const std::string& msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return code;
}

#define FLAME_HIP(c, call)                                                        \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail((c), FLAME_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

std::string validate(const flame_params* p) {
  if (!p) return "params is NULL";
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "grid sizes must be >= 1";
  if (p->jmode == FLAME_J_STENCIL && (p->nx < 3 || p->ny < 3 || p->nz < 3))
    return "the stencil current needs every grid size >= 3";
  const double cells = static_cast<double>(p->nx) * p->ny * p->nz;
  if (cells >= 1099511627776.0) return "grid too large (nx*ny*nz must be < 2^40)";
  if (p->nz > 65535) return "nz must be <= 65535";
  // kernels address each population and forcing array with 32-bit byte offsets: every array,
  // with its stride padding, must span at most 4 GiB (largest offset 4 GiB minus one value)
  const double vb = p->storage == FLAME_F64 ? 8.0 : p->storage == FLAME_F32 ? 4.0 : 2.0;
  const double fb = p->storage == FLAME_F64 ? 8.0 : 4.0;
  const bool forced = p->force_u || p->force_b;
  if (cells >= 4294967296.0 || static_cast<double>(population_stride(*p)) * vb > 4294967296.0 ||
      (forced && cells * fb > 4294967296.0))
    return "grid too large: each population / forcing array must fit in 4 GiB";
  if (!(p->nu > 0) || !isfinite(p->nu)) return "nu must be finite and > 0";
  if (!(p->eta > 0) || !isfinite(p->eta)) return "eta must be finite and > 0";
  if (!(p->d_i >= 0) || !isfinite(p->d_i)) return "d_i must be finite and >= 0";
  for (int i = 0; i < 3; ++i)
    if (!isfinite(p->b0[i])) return "b0 must be finite";
  if (p->storage != FLAME_F64 && p->storage != FLAME_F32 && p->storage != FLAME_F16)
    return "unknown storage";
  if (p->jmode != FLAME_J_MOMENT && p->jmode != FLAME_J_STENCIL) return "unknown jmode";
  if (p->layout != FLAME_LAYOUT_AB && p->layout != FLAME_LAYOUT_AA) return "unknown layout";
  if (p->collision != FLAME_COLLISION_CENTRAL && p->collision != FLAME_COLLISION_BGK) return "unknown collision";
  if (p->magnetic != FLAME_MAGNETIC_HALL && p->magnetic != FLAME_MAGNETIC_EMHD) return "unknown magnetic model";
  if (p->fluid_lattice != FLAME_FLUID_D3Q27 && p->fluid_lattice != FLAME_FLUID_D3Q19) return "unknown fluid lattice";
  if (p->magnetic_lattice != FLAME_MAGNETIC_D3Q7 && p->magnetic_lattice != FLAME_MAGNETIC_D3Q15 &&
      p->magnetic_lattice != FLAME_MAGNETIC_D3Q27)
    return "unknown magnetic lattice";
  return "";
}

// Valid parameters whose combination is not built ("" if it is).
std::string unsupported(const flame_params* p) {
  if (lattice_variant(*p) && p->jmode != FLAME_J_MOMENT)
    return "the lattice variants run the moment route of J only";
  if (p->fluid_lattice == FLAME_FLUID_D3Q19 && p->collision != FLAME_COLLISION_BGK)
    return "the central-moment collision is built on the D3Q27 fluid set; D3Q19 runs the BGK collision";
  return "";
}

size_t values_per_node(const flame_params& p) {
  const size_t one = static_cast<size_t>(fluid_count(p)) + 3 * static_cast<size_t>(mag_count(p));
  if (p.layout == FLAME_LAYOUT_AB) return 2 * one;
  return p.jmode == FLAME_J_STENCIL ? one + 3 * static_cast<size_t>(mag_count(p)) : one;
}

template <typename S>
View<S> make_view(const flame_ctx* c) {
  const SetPtrs s = set_ptrs(c);
  View<S> v;
  v.F = static_cast<const S*>(s.f_src);
  v.G = static_cast<const S*>(s.g_src);
  v.fmode = s.fluid_aa ? (c->parity == 1 ? 1 : 0) : 2;
  v.gmode = s.mag_aa ? (c->parity == 1 ? 1 : 0) : 2;
  v.nx = c->p.nx;
  v.ny = c->p.ny;
  v.nz = c->p.nz;
  v.n = c->n;
  v.stride = c->stride;
  return v;
}

template <typename S>
AuxArgs<S> make_aux(const flame_ctx* c) {
  using R = typename Enc<S>::R;
  AuxArgs<S> a;
  a.v = make_view<S>(c);
  a.force_u = static_cast<const R*>(c->p.force_u);
  a.force_b = static_cast<const R*>(c->p.force_b);
  for (int i = 0; i < 3; ++i) a.b0[i] = c->p.b0[i];
  a.alpha = c->p.d_i;
  a.omega_b = c->omega_b;
  a.stencil = c->p.jmode == FLAME_J_STENCIL;
  a.emhd = c->p.magnetic == FLAME_MAGNETIC_EMHD;
  return a;
}

// Rest state for full-value copies; all zeros for deviation copies.
Rest make_rest(const flame_ctx* c, int32_t deviations) {
  Rest r;
  for (int i = 0; i < 27; ++i) r.f[i] = deviations ? 0.0 : c->frest[i];
  for (int i = 0; i < 3; ++i) r.b0[i] = deviations ? 0.0 : c->p.b0[i];
  return r;
}

Placement make_placement(const flame_ctx* c) {
  const SetPtrs s = set_ptrs(c);
  Placement at;
  at.fpull = !s.fluid_aa;
  at.gpull = !s.mag_aa;
  at.nx = c->p.nx;
  at.ny = c->p.ny;
  at.nz = c->p.nz;
  return at;
}

unsigned blocks_for(size_t n, int threads) { return static_cast<unsigned>((n + threads - 1) / threads); }

// Dispatch a callable templated on the storage type.
template <typename Fn>
hipError_t by_storage(const flame_ctx* c, Fn&& fn) {
  switch (c->p.storage) {
    case FLAME_F64: return fn(double{});
    case FLAME_F32: return fn(float{});
    default: return fn(_Float16{});
  }
}

__global__ void max_field_kernel(const double* b, double b0x, double b0y, double b0z, size_t n, double* out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const double x = b0x + b[k], y = b0y + b[n + k], z = b0z + b[2 * n + k];
    m = fmax(m, sqrt(x * x + y * y + z * z));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (unsigned s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// Device address of this device's copy of the scratch array, looked up once per device (with that
// device current) and kept for the process.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

// Lattice sound speed c_s = 1/sqrt(3): the flame_reduce guard on max |u|.
constexpr double kSoundSpeed = 0.57735026918962576;

// The reductions of the current state: block partials into partials (c->red_blocks x FLAME_NRED
// doubles), merged in a fixed order into out (FLAME_NRED doubles, device). Asynchronous.
hipError_t launch_reduce(const flame_ctx* c, double* partials, double* out) {
  hipError_t e = lattice_variant(c->p) ? variant_launch_reduce(c, partials) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(reduce_kernel<S>, dim3(c->red_blocks), dim3(kRedThreads), 0, c->stream, make_aux<S>(c),
                       partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_merge_kernel, dim3(1), dim3(64), 0, c->stream, partials, c->red_blocks,
                     static_cast<double>(c->n), out);
  return hipGetLastError();
}

}  // namespace

namespace flame {
SetPtrs set_ptrs(const flame_ctx* c) {
  const size_t vb = value_bytes(c->p.storage);
  const size_t n = c->stride;
  const size_t nf = fluid_count(c->p), ng = 3 * static_cast<size_t>(mag_count(c->p));
  char* base = static_cast<char*>(c->storage);
  SetPtrs s{};
  if (c->p.layout == FLAME_LAYOUT_AB) {
    char* F0 = base;
    char* F1 = base + nf * n * vb;
    char* G0 = base + 2 * nf * n * vb;
    char* G1 = G0 + ng * n * vb;
    s.f_src = c->cur ? F1 : F0;
    s.f_dst = c->cur ? F0 : F1;
    s.g_src = c->cur ? G1 : G0;
    s.g_dst = c->cur ? G0 : G1;
    s.fluid_aa = false;
    s.mag_aa = false;
  } else {
    s.f_src = s.f_dst = base;
    s.fluid_aa = true;
    char* G0 = base + nf * n * vb;
    if (c->p.jmode == FLAME_J_STENCIL) {
      char* G1 = G0 + ng * n * vb;
      s.g_src = c->cur ? G1 : G0;
      s.g_dst = c->cur ? G0 : G1;
      s.mag_aa = false;
    } else {
      s.g_src = s.g_dst = G0;
      s.mag_aa = true;
    }
  }
  return s;
}
}  // namespace flame

extern "C" {

flame_status flame_rest_populations(const flame_params* p, double* f_rest, double* g_rest) {
  if (!p) return FLAME_E_INVAL;
  if (lattice_variant(*p)) {
    if (!validate(p).empty()) return FLAME_E_INVAL;
    variant_rest(*p, f_rest, g_rest);
    return FLAME_OK;
  }
  // f^mhd(0)(1, 0, b0) = w_i + (w_i / 2 c_s^4) M(b0) : (c c - c_s^2 I), M = |b0|^2/2 I - b0 b0,
  // with M : (c c - I/3) = |b0|^2/2 (|c|^2 - 1/3) - (b0 . c)^2
  const double* B0 = p->b0;
  const double b2 = B0[0] * B0[0] + B0[1] * B0[1] + B0[2] * B0[2];
  if (f_rest)
    for (int i = 0; i < 27; ++i) {
      const double cb = cq(i, 0) * B0[0] + cq(i, 1) * B0[1] + cq(i, 2) * B0[2];
      f_rest[i] = wq(i) + wq(i) * 4.5 * (0.5 * b2 * (speed2q(i) - 1.0 / 3.0) - cb * cb);
    }
  if (g_rest)
    for (int i = 0; i < 7; ++i)
      for (int c = 0; c < 3; ++c) g_rest[i * 3 + c] = wm(i) * B0[c];
  return FLAME_OK;
}

size_t flame_storage_bytes(const flame_params* p) {
  if (!validate(p).empty() || !unsupported(p).empty()) return 0;
  return values_per_node(*p) * value_bytes(p->storage) * population_stride(*p);
}

flame_status flame_init(const flame_params* p, const double* u, const double* b, const double* grad_u,
                        const double* grad_b, void* storage, size_t storage_bytes, void* hip_stream,
                        flame_ctx** out) {
  g_init_error.clear();
  if (!out) return fail(nullptr, FLAME_E_INVAL, "out is NULL");
  *out = nullptr;
  const std::string bad = validate(p);
  if (!bad.empty()) return fail(nullptr, FLAME_E_INVAL, bad);
  const std::string not_built = unsupported(p);
  if (!not_built.empty()) return fail(nullptr, FLAME_E_UNSUPPORTED, not_built);
  if (!u || !b) return fail(nullptr, FLAME_E_INVAL, "u and b must be given");
  if (!storage) return fail(nullptr, FLAME_E_INVAL, "storage is NULL");
  if (reinterpret_cast<uintptr_t>(storage) % 256 != 0) return fail(nullptr, FLAME_E_INVAL, "storage must be 256-byte aligned");
  const size_t need = flame_storage_bytes(p);
  if (storage_bytes < need)
    return fail(nullptr, FLAME_E_INVAL, "storage too small: need " + std::to_string(need) + " bytes");
  flame_ctx* c = new (std::nothrow) flame_ctx;
  if (!c) return fail(nullptr, FLAME_E_NOMEM, "context allocation failed");
  c->p = *p;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->n = static_cast<size_t>(p->nx) * p->ny * p->nz;
  c->stride = population_stride(*p);
  c->storage = storage;
  c->omega = 1.0 / (3.0 * p->nu + 0.5);
  c->omega_b = 1.0 / (4.0 * p->eta + 0.5);
  // launch-shape tuning (multiples of 64 threads per row block; any positive plane count)
  if (const char* v = getenv("FLAME_ZCHUNK_PLANES")) c->zchunk = std::max(0, atoi(v));
  if (const char* v = getenv("FLAME_ROW_THREADS")) c->row_tx = std::min(std::max(0, atoi(v)) / 64 * 64, kRowThreadsMax);
  if (const char* v = getenv("FLAME_GLOBAL_ADDRESSING")) c->global_addr = atoi(v) != 0;
  const double* B0 = p->b0;
  flame_rest_populations(p, c->frest, nullptr);   // q <= 27 values
  auto bail = [&](flame_status code) {
    g_init_error = c->err;
    delete c;
    return code;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    c->err = "hipGetDevice failed (no HIP device?)";
    return bail(FLAME_E_HIP);
  }
  {
    const hipError_t e = scratch_address(c->device, &c->scratch);
    if (e != hipSuccess) {
      c->err = std::string("hipGetSymbolAddress of the reduction scratch: ") + hipGetErrorString(e);
      return bail(FLAME_E_HIP);
    }
  }
  c->red_blocks = static_cast<int>(std::min<size_t>(kRedBlocksMax, blocks_for(c->n, kRedThreads)));
  // block partials of the reductions plus one row for their merged results
  if (hipMalloc(&c->red_partials, sizeof(double) * FLAME_NRED * (std::max(c->red_blocks, 1) + 1)) != hipSuccess) {
    c->err = "hipMalloc of reduction scratch failed";
    return bail(FLAME_E_NOMEM);
  }
  // initial state into the canonical slots of copy 0
  const SetPtrs s = set_ptrs(c);
  hipError_t e = lattice_variant(*p) ? variant_launch_init(c, u, b, grad_u, grad_b) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Enc<S>::R;
    InitArgs<S> a;
    a.F = static_cast<S*>(s.f_src);
    a.G = static_cast<S*>(s.g_src);
    a.u = u;
    a.b = b;
    a.gu = grad_u;
    a.gb = grad_b;
    a.force_u = static_cast<const R*>(p->force_u);
    a.force_b = static_cast<const R*>(p->force_b);
    for (int i = 0; i < 3; ++i) a.b0[i] = B0[i];
    a.omega = c->omega;
    a.omega_b = c->omega_b;
    a.alpha = p->d_i;
    a.noneq = p->init_noneq;
    a.emhd = p->magnetic == FLAME_MAGNETIC_EMHD;
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.n = c->n;
    a.stride = c->stride;
    a.at = make_placement(c);
    hipLaunchKernelGGL(init_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream, a);
    return hipGetLastError();
  });
  if (e != hipSuccess) {
    c->err = std::string("init kernel: ") + hipGetErrorString(e);
    return bail(FLAME_E_HIP);
  }
  // advisory CFL number from max |B| of the initial field
  const int mb = static_cast<int>(std::min<size_t>(1024, blocks_for(c->n, 256)));
  hipLaunchKernelGGL(max_field_kernel, dim3(mb), dim3(256), 0, c->stream, b, B0[0], B0[1], B0[2], c->n,
                     c->red_partials);
  double host[1024];
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(host, c->red_partials, sizeof(double) * mb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("initial field maximum: ") + hipGetErrorString(e);
    return bail(FLAME_E_HIP);
  }
  double bmax = 0;
  for (int i = 0; i < mb; ++i) bmax = std::max(bmax, host[i]);
  c->cfl = M_PI * p->d_i * bmax;
  *out = c;
  return c->cfl > 1.0 ? FLAME_W_CFL : FLAME_OK;
}

flame_status flame_step(flame_ctx* c, int64_t nsteps) {
  if (!c) return FLAME_E_INVAL;
  if (nsteps < 0) return fail(c, FLAME_E_INVAL, "nsteps must be >= 0");
  const bool two_f = c->p.layout == FLAME_LAYOUT_AB;
  const bool two_g = mag_two_lattice(c->p);
  for (int64_t s = 0; s < nsteps; ++s) {
    const SetPtrs ptr = set_ptrs(c);
    hipError_t e = launch_step(c, ptr, c->stride, nullptr);
    if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("step kernel: ") + hipGetErrorString(e));
    if (two_f || two_g) c->cur ^= 1;
    if (!two_f || !two_g) c->parity ^= 1;
    c->steps += 1;
  }
  return FLAME_OK;
}

flame_status flame_moments(flame_ctx* c, double* rho, double* u, double* b, double* j, double* divb) {
  if (!c) return FLAME_E_INVAL;
  hipError_t e = lattice_variant(c->p) ? variant_launch_moments(c, rho, u, b, j, divb) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(moments_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream,
                       make_aux<S>(c), rho, u, b, j, divb);
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("moments kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

flame_status flame_reduce(flame_ctx* c, double* out) {
  if (!c || !out) return c ? fail(c, FLAME_E_INVAL, "out is NULL") : FLAME_E_INVAL;
  // block partials, then the merged results behind them in the same scratch
  double* merged = c->red_partials + static_cast<size_t>(c->red_blocks) * FLAME_NRED;
  hipError_t e = launch_reduce(c, c->red_partials, merged);
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("reduce kernel: ") + hipGetErrorString(e));
  FLAME_HIP(c, hipMemcpyAsync(out, merged, sizeof(double) * FLAME_NRED, hipMemcpyDeviceToHost, c->stream));
  FLAME_HIP(c, hipStreamSynchronize(c->stream));
  if (out[8] > 0) return fail(c, FLAME_E_NONFINITE, "non-finite populations at " + std::to_string(out[8]) + " nodes");
  if (out[6] >= kSoundSpeed)
    return fail(c, FLAME_E_UNSTABLE, "max |u| = " + std::to_string(out[6]) + " reached the lattice sound speed");
  return FLAME_OK;
}

flame_status flame_reduce_noalloc(flame_ctx* c, double* out) {
  if (!c || !out) return c ? fail(c, FLAME_E_INVAL, "out is NULL") : FLAME_E_INVAL;
  if (!c->scratch) return fail(c, FLAME_E_HIP, "the reduction scratch of this device was not found at init");
  if (c->red_blocks < 1 || c->red_blocks > kRedBlocksMax)
    return fail(c, FLAME_E_INVAL, "reduction needs " + std::to_string(c->red_blocks) +
                                      " block partials; the static scratch holds " + std::to_string(kRedBlocksMax));
  const hipError_t e = launch_reduce(c, c->scratch, out);
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("reduce kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

}  // extern "C"

namespace {

// Energy (k2 = 0) or dissipation (k2 = 1) shell spectrum of u or B, summed over components.
flame_status shell_spectrum(flame_ctx* c, int32_t field, int32_t nshells, int k2, double* e_k) {
  if (!c) return FLAME_E_INVAL;
  if (field != 0 && field != 1) return fail(c, FLAME_E_INVAL, "field must be 0 (u) or 1 (B)");
  if (nshells < 1 || nshells > kSpecShellsMax) return fail(c, FLAME_E_INVAL, "nshells out of range");
  if (!e_k) return fail(c, FLAME_E_INVAL, "e_k is NULL");
  const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
  const size_t nh = static_cast<size_t>(nz) * ny * (nx / 2 + 1);
  // each buffer is checked on its own, and a failed allocation leaves its pointer null, so a call
  // after an out-of-memory failure allocates again instead of launching on a missing buffer
  if (!c->spec_real && hipMalloc(&c->spec_real, sizeof(double) * c->n) != hipSuccess) {
    c->spec_real = nullptr;
    (void)hipGetLastError();  // clear the allocation error so later launch checks do not see it
    return fail(c, FLAME_E_NOMEM, "spectrum: device workspace");
  }
  if (!c->spec_cplx && hipMalloc(&c->spec_cplx, sizeof(hipfftDoubleComplex) * nh) != hipSuccess) {
    c->spec_cplx = nullptr;
    (void)hipGetLastError();  // clear the allocation error so later launch checks do not see it
    return fail(c, FLAME_E_NOMEM, "spectrum: device workspace");
  }
  if (!c->plan_ok) {
    if (hipfftPlan3d(&c->plan, nz, ny, nx, HIPFFT_D2Z) != HIPFFT_SUCCESS)
      return fail(c, FLAME_E_HIP, "hipfftPlan3d failed");
    c->plan_ok = true;
    if (hipfftSetStream(c->plan, c->stream) != HIPFFT_SUCCESS) return fail(c, FLAME_E_HIP, "hipfftSetStream failed");
  }
  const int blocks = static_cast<int>(std::min<size_t>(kBinBlocksMax, blocks_for(nh, kBinThreads)));
  if (!c->spec_partials || c->spec_blocks != blocks || c->spec_nshells < nshells) {
    if (c->spec_partials) FLAME_HIP(c, hipFree(c->spec_partials));
    c->spec_partials = nullptr;
    c->spec_blocks = 0;
    c->spec_nshells = 0;
    // block partials plus one row for their merged sums
    if (hipMalloc(&c->spec_partials, sizeof(double) * (static_cast<size_t>(blocks) + 1) * nshells) != hipSuccess) {
      c->spec_partials = nullptr;
      (void)hipGetLastError();  // clear the allocation error so later launch checks do not see it
      return fail(c, FLAME_E_NOMEM, "spectrum: device workspace");
    }
    c->spec_blocks = blocks;
    c->spec_nshells = nshells;
  }
  double* merged = c->spec_partials + static_cast<size_t>(blocks) * nshells;
  std::vector<double> host(static_cast<size_t>(nshells));
  for (int s = 0; s < nshells; ++s) e_k[s] = 0.0;
  const double norm2 = 1.0 / (static_cast<double>(c->n) * static_cast<double>(c->n));
  for (int comp = 0; comp < 3; ++comp) {
    hipError_t e = lattice_variant(c->p) ? variant_launch_component(c, field, comp, c->spec_real)
                                         : by_storage(c, [&](auto tag) {
      using S = decltype(tag);
      hipLaunchKernelGGL(field_component_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream,
                         make_aux<S>(c), field, comp, c->spec_real);
      return hipGetLastError();
    });
    if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("field kernel: ") + hipGetErrorString(e));
    if (hipfftExecD2Z(c->plan, c->spec_real, static_cast<hipfftDoubleComplex*>(c->spec_cplx)) != HIPFFT_SUCCESS)
      return fail(c, FLAME_E_HIP, "hipfftExecD2Z failed");
    hipLaunchKernelGGL(shell_bin_kernel, dim3(blocks), dim3(kBinThreads), sizeof(double) * nshells, c->stream,
                       static_cast<const hipfftDoubleComplex*>(c->spec_cplx), nx, ny, nz, nshells, norm2, k2,
                       c->spec_partials);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(bin_merge_kernel, dim3(blocks_for(static_cast<size_t>(nshells), 256), 1), dim3(256), 0,
                         c->stream, c->spec_partials, blocks, nshells, merged);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(host.data(), merged, sizeof(double) * nshells, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("spectrum: ") + hipGetErrorString(e));
    for (int s = 0; s < nshells; ++s) e_k[s] += host[s];
  }
  return FLAME_OK;
}

}  // namespace

extern "C" {

flame_status flame_spectrum(flame_ctx* c, int32_t field, int32_t nshells, double* e_k) {
  return shell_spectrum(c, field, nshells, 0, e_k);
}

flame_status flame_dissipation_spectrum(flame_ctx* c, int32_t field, int32_t nshells, double* d_k) {
  return shell_spectrum(c, field, nshells, 1, d_k);
}

}  // extern "C"

namespace {

// Device buffers of one energy-transfer evaluation, released on every return once the work
// queued on the stream (which may still use them on an error path) has finished.
struct TransferScratch {
  hipStream_t stream;
  double* real = nullptr;              // U(3) B(3) J(3), a work field, the advection product
  hipfftDoubleComplex* cplx = nullptr; // u_hat(3) B_hat(3), a work spectrum
  double* partials = nullptr;          // 4 terms x blocks x nshells
  explicit TransferScratch(hipStream_t s) : stream(s) {}
  ~TransferScratch() {
    (void)hipStreamSynchronize(stream);
    if (real) (void)hipFree(real);
    if (cplx) (void)hipFree(cplx);
    if (partials) (void)hipFree(partials);
  }
};

flame_status energy_transfer(flame_ctx* c, int32_t nshells, double* t_adv, double* t_lor, double* t_ind,
                             double* t_hall) {
  if (!c) return FLAME_E_INVAL;
  if (nshells < 1 || nshells > kSpecShellsMax) return fail(c, FLAME_E_INVAL, "nshells out of range");
  if (!t_adv || !t_lor || !t_ind) return fail(c, FLAME_E_INVAL, "an output array is NULL");
  const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
  const size_t n = c->n;
  const size_t nh = static_cast<size_t>(nz) * ny * (nx / 2 + 1);
  if (!c->plan_ok) {
    if (hipfftPlan3d(&c->plan, nz, ny, nx, HIPFFT_D2Z) != HIPFFT_SUCCESS)
      return fail(c, FLAME_E_HIP, "hipfftPlan3d failed");
    c->plan_ok = true;
    if (hipfftSetStream(c->plan, c->stream) != HIPFFT_SUCCESS) return fail(c, FLAME_E_HIP, "hipfftSetStream failed");
  }
  if (!c->plan_inv_ok) {
    if (hipfftPlan3d(&c->plan_inv, nz, ny, nx, HIPFFT_Z2D) != HIPFFT_SUCCESS)
      return fail(c, FLAME_E_HIP, "hipfftPlan3d (inverse) failed");
    c->plan_inv_ok = true;
    if (hipfftSetStream(c->plan_inv, c->stream) != HIPFFT_SUCCESS)
      return fail(c, FLAME_E_HIP, "hipfftSetStream failed");
  }
  const int blocks = static_cast<int>(std::min<size_t>(kBinBlocksMax, blocks_for(nh, kBinThreads)));
  TransferScratch w(c->stream);
  if (hipMalloc(&w.real, sizeof(double) * 11 * n) != hipSuccess) w.real = nullptr;
  if (w.real && hipMalloc(&w.cplx, sizeof(hipfftDoubleComplex) * 7 * nh) != hipSuccess) w.cplx = nullptr;
  // 4 terms of block partials, then the 4 merged rows
  if (w.cplx && hipMalloc(&w.partials, sizeof(double) * 4 * (static_cast<size_t>(blocks) + 1) * nshells) != hipSuccess)
    w.partials = nullptr;
  if (!w.partials) {
    (void)hipGetLastError();  // clear the allocation error so later launch checks do not see it
    return fail(c, FLAME_E_NOMEM, "energy transfer: device workspace");
  }
  double* U = w.real;
  double* B = w.real + 3 * n;
  double* J = w.real + 6 * n;
  double* work = w.real + 9 * n;
  double* adv = w.real + 10 * n;
  hipfftDoubleComplex* Uh = w.cplx;
  hipfftDoubleComplex* Bh = w.cplx + 3 * nh;
  hipfftDoubleComplex* spec = w.cplx + 6 * nh;
  const unsigned gn = blocks_for(n, 256), gh = blocks_for(nh, 256);
  hipError_t e = lattice_variant(c->p) ? variant_launch_moments(c, nullptr, U, B, J, nullptr) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(moments_kernel<S>, dim3(gn), dim3(256), 0, c->stream, make_aux<S>(c), nullptr, U, B, J,
                       nullptr);
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("energy transfer fields: ") + hipGetErrorString(e));
  // forward transforms run on the work copy: the transform may overwrite its input
  auto forward = [&](const double* src, hipfftDoubleComplex* dst) -> bool {
    if (src != work && hipMemcpyAsync(work, src, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return false;
    return hipfftExecD2Z(c->plan, work, dst) == HIPFFT_SUCCESS;
  };
  const double norm2 = 1.0 / (static_cast<double>(n) * static_cast<double>(n));
  auto bin = [&](int kind, int term, const hipfftDoubleComplex* X, int comp, double sign, bool first) {
    hipLaunchKernelGGL(transfer_bin_kernel, dim3(blocks), dim3(kBinThreads), sizeof(double) * nshells, c->stream,
                       kind, X, spec, Bh, comp, sign, nx, ny, nz, nshells, norm2, first ? 1 : 0,
                       w.partials + static_cast<size_t>(term) * blocks * nshells);
    return hipGetLastError() == hipSuccess;
  };
  bool ok = true;
  for (int b = 0; b < 3 && ok; ++b) ok = forward(U + b * n, Uh + b * nh) && forward(B + b * n, Bh + b * nh);
  for (int b = 0; b < 3 && ok; ++b) {
    // (U . grad) U_b, with grad U_b from the inverse transform of i q_a u_hat_b
    for (int a = 0; a < 3 && ok; ++a) {
      hipLaunchKernelGGL(spectral_derivative_kernel, dim3(gh), dim3(256), 0, c->stream, Uh + b * nh, nx, ny, nz, a,
                         1.0 / static_cast<double>(n), spec);
      ok = hipGetLastError() == hipSuccess && hipfftExecZ2D(c->plan_inv, spec, work) == HIPFFT_SUCCESS;
      if (ok) {
        hipLaunchKernelGGL(product_accumulate_kernel, dim3(gn), dim3(256), 0, c->stream, adv, U + a * n, work, n,
                           a == 0 ? 1 : 0);
        ok = hipGetLastError() == hipSuccess;
      }
    }
    ok = ok && forward(adv, spec) && bin(0, 0, Uh + b * nh, b, 1.0, b == 0);
    // Lorentz force (J x B)_b; the Hall term takes the same transform against conj(B_hat) x q
    if (ok) {
      hipLaunchKernelGGL(cross_component_kernel, dim3(gn), dim3(256), 0, c->stream, J, B, b, n, work);
      ok = hipGetLastError() == hipSuccess && forward(work, spec) && bin(0, 1, Uh + b * nh, b, -1.0, b == 0);
      if (ok && t_hall) ok = bin(1, 3, nullptr, b, -c->p.d_i, b == 0);
    }
    // induction: (U x B)_b, binned against conj(B_hat) x q
    if (ok) {
      hipLaunchKernelGGL(cross_component_kernel, dim3(gn), dim3(256), 0, c->stream, U, B, b, n, work);
      ok = hipGetLastError() == hipSuccess && forward(work, spec) && bin(1, 2, nullptr, b, 1.0, b == 0);
    }
  }
  const int terms = t_hall ? 4 : 3;
  double* merged = w.partials + static_cast<size_t>(4) * blocks * nshells;
  if (ok) {
    hipLaunchKernelGGL(bin_merge_kernel, dim3(blocks_for(static_cast<size_t>(nshells), 256), terms), dim3(256), 0,
                       c->stream, w.partials, blocks, nshells, merged);
    ok = hipGetLastError() == hipSuccess;
  }
  std::vector<double> host(static_cast<size_t>(terms) * nshells);
  if (ok) ok = hipMemcpyAsync(host.data(), merged, sizeof(double) * host.size(), hipMemcpyDeviceToHost,
                              c->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) {
    const hipError_t last = hipGetLastError();
    return fail(c, FLAME_E_HIP, std::string("energy transfer: a transform, copy or kernel launch failed (") +
                                    hipGetErrorString(last) + ")");
  }
  double* outs[4] = {t_adv, t_lor, t_ind, t_hall};
  for (int t = 0; t < terms; ++t)
    for (int s = 0; s < nshells; ++s) outs[t][s] = host[static_cast<size_t>(t) * nshells + s];
  return FLAME_OK;
}

}  // namespace

extern "C" {

flame_status flame_energy_transfer(flame_ctx* c, int32_t nshells, double* t_adv, double* t_lor, double* t_ind,
                                   double* t_hall) {
  return energy_transfer(c, nshells, t_adv, t_lor, t_ind, t_hall);
}

flame_status flame_get_populations(flame_ctx* c, double* dst, int32_t deviations) {
  if (!c || !dst) return c ? fail(c, FLAME_E_INVAL, "dst is NULL") : FLAME_E_INVAL;
  hipError_t e = lattice_variant(c->p) ? variant_launch_get(c, deviations, dst) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(get_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream, make_view<S>(c),
                       make_rest(c, deviations), dst);
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("get kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

flame_status flame_set_populations(flame_ctx* c, const double* src, int32_t deviations) {
  if (!c || !src) return c ? fail(c, FLAME_E_INVAL, "src is NULL") : FLAME_E_INVAL;
  c->cur = 0;
  c->parity = 0;
  c->steps = 0;
  const SetPtrs s = set_ptrs(c);
  hipError_t e = lattice_variant(c->p) ? variant_launch_set(c, deviations, src) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(set_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream,
                       static_cast<S*>(s.f_src), static_cast<S*>(s.g_src), c->n, c->stride, make_placement(c),
                       make_rest(c, deviations), src);
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("set kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

flame_status flame_gather(flame_ctx* c, const int64_t* cells, int64_t n, double* out, int32_t deviations) {
  if (!c) return FLAME_E_INVAL;
  if (n < 0 || (n > 0 && (!cells || !out))) return fail(c, FLAME_E_INVAL, "bad gather arguments");
  if (n == 0) return FLAME_OK;
  hipError_t e = lattice_variant(c->p) ? variant_launch_gather(c, deviations, cells, n, out) : by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(gather_kernel<S>, dim3(blocks_for(static_cast<size_t>(n), 256)), dim3(256), 0, c->stream,
                       make_view<S>(c), make_rest(c, deviations), cells, n, out);
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("gather kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

size_t flame_trace_bytes(const flame_ctx* c) {
  return c && reverse_mode_built(c->p) ? 48 * c->n * value_bytes(c->p.storage) : 0;
}

flame_status flame_trace_export(flame_ctx* c, void* lat) {
  if (!c) return FLAME_E_INVAL;
  if (c->p.layout != FLAME_LAYOUT_AA || c->p.jmode != FLAME_J_MOMENT)
    return fail(c, FLAME_E_UNSUPPORTED, "trace export is available on the moment route with the AA layout only");
  if (!reverse_mode_built(c->p))
    return fail(c, FLAME_E_UNSUPPORTED, "reverse mode is built for the paper's model and velocity sets only");
  if (!lat) return fail(c, FLAME_E_INVAL, "lat is NULL");
  hipError_t e = by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(export_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream, make_view<S>(c),
                       static_cast<S*>(lat));
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("export kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

flame_status flame_adjoint_fields(flame_ctx* c, const double* dl_du, const double* dl_db, void* lam) {
  if (!c) return FLAME_E_INVAL;
  if (!reverse_mode_built(c->p))
    return fail(c, FLAME_E_UNSUPPORTED, "reverse mode is built for the paper's model and velocity sets only");
  if (!lam) return fail(c, FLAME_E_INVAL, "lam is NULL");
  hipError_t e = by_storage(c, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Enc<S>::R;
    hipLaunchKernelGGL(adjoint_fields_kernel<S>, dim3(blocks_for(c->n, 256)), dim3(256), 0, c->stream,
                       make_view<S>(c), static_cast<const R*>(c->p.force_u), dl_du, dl_db, static_cast<R*>(lam));
    return hipGetLastError();
  });
  if (e != hipSuccess) return fail(c, FLAME_E_HIP, std::string("field adjoint kernel: ") + hipGetErrorString(e));
  return FLAME_OK;
}

int64_t flame_step_count(const flame_ctx* c) { return c ? c->steps : -1; }

double flame_cfl_number(const flame_ctx* c) { return c ? c->cfl : 0.0; }

const char* flame_last_error(const flame_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void flame_destroy(flame_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->plan_ok) hipfftDestroy(c->plan);
  if (c->plan_inv_ok) hipfftDestroy(c->plan_inv);
  if (c->red_partials) (void)hipFree(c->red_partials);
  if (c->spec_real) (void)hipFree(c->spec_real);
  if (c->spec_cplx) (void)hipFree(c->spec_cplx);
  if (c->spec_partials) (void)hipFree(c->spec_partials);
  delete c;
}

}  // extern "C"
