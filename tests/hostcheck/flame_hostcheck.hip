// Host build of the library's per-node arithmetic (test infrastructure): lets the CPU test
// suite check the kernels' collision and its reverse pass against the oracle without a GPU.
#include "../../paper_2212_11024_amd/csrc/flame_device.h"
#include "../../paper_2212_11024_amd/csrc/flame_internal.h"
#include "../../paper_2212_11024_amd/csrc/flame_lattice.h"

using namespace flame;

namespace {
PhysConst<double> consts(const double* p) {
  PhysConst<double> k;
  k.omega = p[0];
  k.omega_b = p[1];
  k.alpha = p[2];
  k.b0[0] = p[3];
  k.b0[1] = p[4];
  k.b0[2] = p[5];
  return k;
}
}  // namespace

extern "C" {

// One node's collision on deviations. params = {omega, omega_b, alpha, b0x, b0y, b0z}.
// mode bit 0 set: J from the moments (J_in ignored); else J = J_in. J_out receives the J used.
// mode bit 1 set: the fluid directions formed in the grouped (c_x, c_y) order.
void hc_collide(int mode, const double* f_in, const double* g_in, const double* Fin, const double* Sin,
                const double* J_in, const double* params, double* f_out, double* g_out, double* J_out) {
  const PhysConst<double> k = consts(params);
  double f[kQ], g[kM], F[3], S[3];
  for (int i = 0; i < kQ; ++i) f[i] = f_in[i];
  for (int i = 0; i < kM; ++i) g[i] = g_in[i];
  for (int c = 0; c < 3; ++c) { F[c] = Fin[c]; S[c] = Sin[c]; }
  const FluidMoments<double> m = fluid_moments(f);
  const double rho = 1.0 + m.drho;
  const double U[3] = {(m.jx + 0.5 * F[0]) / rho, (m.jy + 0.5 * F[1]) / rho, (m.jz + 0.5 * F[2]) / rho};
  double b[3], lam[3][3];
  magnetic_moments(g, b, lam);
  for (int c = 0; c < 3; ++c) b[c] += 0.5 * S[c];
  const double B[3] = {k.b0[0] + b[0], k.b0[1] + b[1], k.b0[2] + b[2]};
  double J[3];
  if (mode & 1) current_from_moments(lam, U, B, k.alpha, k.omega_b, J);
  else for (int c = 0; c < 3; ++c) J[c] = J_in[c];
  const double b0[3] = {k.b0[0], k.b0[1], k.b0[2]};
  if (mode & 2) collide_fluid<double, true>(f, m, rho, U, b, b0, F, k.omega);
  else collide_fluid<double, false>(f, m, rho, U, b, b0, F, k.omega);
  collide_magnetic(g, U, B, b, J, S, k.alpha, k.omega_b);
  for (int i = 0; i < kQ; ++i) f_out[i] = f[i];
  for (int i = 0; i < kM; ++i) g_out[i] = g[i];
  for (int c = 0; c < 3; ++c) J_out[c] = J[c];
}

void hc_collide_vjp(int moment, const double* f_in, const double* g_in, const double* Fin, const double* Sin,
                    const double* J_in, const double* params, const double* mf_in, const double* mg_in,
                    double* lf_out, double* lg_out, double* lJ_out) {
  const PhysConst<double> k = consts(params);
  double f[kQ], g[kM], F[3], S[3], J[3], mf[kQ], mg[kM], lf[kQ], lg[kM], lJ[3];
  for (int i = 0; i < kQ; ++i) { f[i] = f_in[i]; mf[i] = mf_in[i]; }
  for (int i = 0; i < kM; ++i) { g[i] = g_in[i]; mg[i] = mg_in[i]; }
  for (int c = 0; c < 3; ++c) { F[c] = Fin[c]; S[c] = Sin[c]; J[c] = J_in[c]; }
  if (moment) collide_vjp<double, true>(f, g, F, S, J, k, mf, mg, lf, lg, lJ);
  else collide_vjp<double, false>(f, g, F, S, J, k, mf, mg, lf, lg, lJ);
  for (int i = 0; i < kQ; ++i) lf_out[i] = lf[i];
  for (int i = 0; i < kM; ++i) lg_out[i] = lg[i];
  for (int c = 0; c < 3; ++c) lJ_out[c] = lJ[c];
}

}  // extern "C"

extern "C" {

// Initial deviations of one node. flags = {fluid_noneq, mag_noneq, has_H}.
void hc_init(const double* u_in, const double* b_in, const double* G_in, const double* H_in, const double* Fin,
             const double* Sin, const double* params, const int* flags, double* f_out, double* g_out) {
  const PhysConst<double> k = consts(params);
  double u[3], b[3], G[3][3], H[3][3], F[3], S[3], f[kQ], g[kM];
  for (int a = 0; a < 3; ++a) {
    u[a] = u_in[a]; b[a] = b_in[a]; F[a] = Fin[a]; S[a] = Sin[a];
    for (int c = 0; c < 3; ++c) { G[a][c] = G_in[a * 3 + c]; H[a][c] = H_in[a * 3 + c]; }
  }
  InitFlags fl{flags[0] != 0, flags[1] != 0, flags[2] != 0};
  init_node(u, b, G, H, F, S, k, fl, f, g);
  for (int i = 0; i < kQ; ++i) f_out[i] = f[i];
  for (int i = 0; i < kM; ++i) g_out[i] = g[i];
}

void hc_init_vjp(const double* u_in, const double* b_in, const double* G_in, const double* H_in, const double* Fin,
                 const double* params, const int* flags, const double* lf_in, const double* lg_in, double* gu_out,
                 double* gb_out, double* gG_out, double* gH_out) {
  const PhysConst<double> k = consts(params);
  double u[3], b[3], G[3][3], H[3][3], F[3], lf[kQ], lg[kM], gu[3], gb[3], gG[3][3], gH[3][3];
  for (int a = 0; a < 3; ++a) {
    u[a] = u_in[a]; b[a] = b_in[a]; F[a] = Fin[a];
    for (int c = 0; c < 3; ++c) { G[a][c] = G_in[a * 3 + c]; H[a][c] = H_in[a * 3 + c]; }
  }
  for (int i = 0; i < kQ; ++i) lf[i] = lf_in[i];
  for (int i = 0; i < kM; ++i) lg[i] = lg_in[i];
  InitFlags fl{flags[0] != 0, flags[1] != 0, flags[2] != 0};
  init_node_vjp(u, b, G, H, F, k, fl, lf, lg, gu, gb, gG, gH);
  for (int a = 0; a < 3; ++a) {
    gu_out[a] = gu[a]; gb_out[a] = gb[a];
    for (int c = 0; c < 3; ++c) { gG_out[a * 3 + c] = gG[a][c]; gH_out[a * 3 + c] = gH[a][c]; }
  }
}

}  // extern "C"

extern "C" {

// One node's collision on a lattice variant, on deviations (the arithmetic of the variant step).
// fq = 27 or 19 fluid velocities, mq = 7, 15 or 27 magnetic; params as for hc_collide.
int hc_variant_collide(int fq, int mq, int bgk, int emhd, const double* f_in, const double* g_in, const double* Fin,
                       const double* Sin, const double* params, double* f_out, double* g_out) {
  const PhysConst<double> k = consts(params);
  const double F[3] = {Fin[0], Fin[1], Fin[2]}, S[3] = {Sin[0], Sin[1], Sin[2]};
  auto run = [&](auto fltag, auto mltag) {
    using FL = decltype(fltag);
    using ML = decltype(mltag);
    double f[FL::q], g[ML::m * 3];
    for (int i = 0; i < FL::q; ++i) f[i] = f_in[i];
    for (int i = 0; i < ML::m * 3; ++i) g[i] = g_in[i];
    if (bgk && emhd) lattice::variant_node<FL, ML, true, true>(f, g, F, S, k);
    else if (bgk) lattice::variant_node<FL, ML, true, false>(f, g, F, S, k);
    else if (emhd) lattice::variant_node<FL, ML, false, true>(f, g, F, S, k);
    else lattice::variant_node<FL, ML, false, false>(f, g, F, S, k);
    for (int i = 0; i < FL::q; ++i) f_out[i] = f[i];
    for (int i = 0; i < ML::m * 3; ++i) g_out[i] = g[i];
  };
  auto by_mag = [&](auto fl) {
    if (mq == 7) run(fl, lattice::Mag<7>{});
    else if (mq == 15) run(fl, lattice::Mag<15>{});
    else run(fl, lattice::Mag<27>{});
  };
  if (fq == 19) {
    if (!bgk) return -1;
    by_mag(lattice::Fluid<19>{});
  } else {
    by_mag(lattice::Fluid<27>{});
  }
  return 0;
}

// Launch policy of the library (host logic): whether the node-local step may address the
// arrays of an nx x ny x nz grid of this storage through buffer resources (arith: the launch
// also reads forcing or writes a saved state), and the threads per row block it launches for a
// row of nx nodes with FLAME_ROW_THREADS = row_tx (0: unset).
int hc_buffer_ok(int nx, int ny, int nz, int storage, int arith) {
  flame_params p{};
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.storage = storage;
  return buffer_addressing_ok(p, arith != 0) ? 1 : 0;
}
unsigned hc_row_threads(int nx, int row_tx) {
  flame_ctx c;
  c.p.nx = nx;
  c.row_tx = row_tx;
  return row_threads(&c);
}

}  // extern "C"
