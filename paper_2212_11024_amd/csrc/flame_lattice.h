// Velocity sets and per-node arithmetic of the lattice variants (the D3Q19 fluid set; the D3Q15 /
// D3Q27 magnetic sets), host-and-device so that the CPU test suite can check them against the
// oracle. The readings the paper leaves open (velocity orders, magnetic weights, the D3Q19
// equilibrium and force term) are stated in include/flame.h next to the FLAME_FLUID_* /
// FLAME_MAGNETIC_* values.
#pragma once

#include "flame_device.h"

namespace flame {
namespace lattice {

// ------------------------------------------------------------------ velocity sets
// Fluid sets: c(i, a), weights, opposite, and the FP16 storage scale (a power of two near 1 / w,
// exact in every format).
template <int Q>
struct Fluid;

template <>
struct Fluid<27> {
  static constexpr int q = 27;
  static FLAME_HD constexpr int c(int i, int a) { return cq(i, a); }
  static FLAME_HD constexpr double w(int i) { return wq(i); }
  static FLAME_HD constexpr int opp(int i) { return oppq(i); }
  static FLAME_HD constexpr int speed2(int i) { return speed2q(i); }
  static FLAME_HD constexpr double f16scale(int i) { return Enc<_Float16>::fscale(i); }
};

// D3Q19: the App. A listing without its corners (directions 0..9 and 14..22 of it).
template <>
struct Fluid<19> {
  static constexpr int q = 19;
  static FLAME_HD constexpr int src(int i) { return i < 10 ? i : i + 4; }
  static FLAME_HD constexpr int c(int i, int a) { return cq(src(i), a); }
  static FLAME_HD constexpr int speed2(int i) { return speed2q(src(i)); }
  static FLAME_HD constexpr double w(int i) {
    return speed2(i) == 0 ? 1.0 / 3.0 : speed2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
  }
  static FLAME_HD constexpr int opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
  static FLAME_HD constexpr double f16scale(int i) { return speed2(i) == 0 ? 4.0 : speed2(i) == 1 ? 16.0 : 32.0; }
};

// Magnetic sets: xi(i, a), weights, opposite, FP16 scale. C^2 = 1/4 for all of them.
template <int M>
struct Mag;

template <>
struct Mag<7> {
  static constexpr int m = 7;
  static FLAME_HD constexpr int xi(int i, int a) { return xim(i, a); }
  static FLAME_HD constexpr double w(int i) { return wm(i); }
  static FLAME_HD constexpr int opp(int i) { return oppm(i); }
  static FLAME_HD constexpr double f16scale(int i) { return Enc<_Float16>::mscale(i); }
};

template <>
struct Mag<15> {
  static constexpr int m = 15;
  static FLAME_HD constexpr int xi(int i, int a) {
    constexpr int8_t t[15][3] = {{0, 0, 0},    {-1, 0, 0},  {0, -1, 0}, {0, 0, -1}, {-1, -1, -1},
                                 {-1, -1, 1},  {-1, 1, -1}, {-1, 1, 1}, {1, 0, 0},  {0, 1, 0},
                                 {0, 0, 1},    {1, 1, 1},   {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    return t[i][a];
  }
  static FLAME_HD constexpr int speed2(int i) { return xi(i, 0) * xi(i, 0) + xi(i, 1) * xi(i, 1) + xi(i, 2) * xi(i, 2); }
  static FLAME_HD constexpr double w(int i) {
    return speed2(i) == 0 ? 5.0 / 12.0 : speed2(i) == 1 ? 1.0 / 12.0 : 1.0 / 96.0;
  }
  static FLAME_HD constexpr int opp(int i) { return i == 0 ? 0 : (i <= 7 ? i + 7 : i - 7); }
  static FLAME_HD constexpr double f16scale(int i) { return speed2(i) == 0 ? 2.0 : speed2(i) == 1 ? 16.0 : 128.0; }
};

template <>
struct Mag<27> {
  static constexpr int m = 27;
  static FLAME_HD constexpr int xi(int i, int a) { return cq(i, a); }
  static FLAME_HD constexpr double w(int i) {
    return speed2q(i) == 0 ? 17.0 / 36.0 : speed2q(i) == 1 ? 1.0 / 18.0 : speed2q(i) == 2 ? 1.0 / 72.0 : 1.0 / 288.0;
  }
  static FLAME_HD constexpr int opp(int i) { return oppq(i); }
  static FLAME_HD constexpr double f16scale(int i) {
    return speed2q(i) == 0 ? 2.0 : speed2q(i) == 1 ? 16.0 : speed2q(i) == 2 ? 64.0 : 256.0;
  }
};

// Storage scale of population i: the FP16 power of two, 1 for FP32 / FP64.
template <typename S, typename L>
FLAME_HD constexpr double fscale(int i) { return sizeof(S) == 2 ? L::f16scale(i) : 1.0; }

// ------------------------------------------------------------------ per-node arithmetic
// Field fluctuation b = sum_i dg_i and Lambda_ab = sum_i xi_ia g_ib (the rest part cancels).
template <typename ML, typename R>
FLAME_HD void mag_moments(const R (&g)[ML::m * 3], R (&b)[3], R (&lam)[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R s = g[c];
#pragma unroll
    for (int i = 1; i < ML::m; ++i) s += g[i * 3 + c];
    b[c] = s;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R s = R(0);
#pragma unroll
      for (int i = 1; i < ML::m; ++i) {
        if (ML::xi(i, a) == 1) s += g[i * 3 + c];
        else if (ML::xi(i, a) == -1) s -= g[i * 3 + c];
      }
      lam[a][c] = s;
    }
}

// Magnetic BGK towards the Hall equilibrium, in deviations dg = g - W b0:
// g*_ic = g_ic - w_B (g_ic - W_i (b_c + 4 sum_a xi_ia E_ac)) + (1 - w_B/2) W_i S_c,
// E_ac = V_a B_c - B_a V_c, V = U - alpha J (eq. gHall_eq with 1/C^2 = 4).
template <typename ML, typename R>
FLAME_HD void collide_mag(R (&g)[ML::m * 3], const R (&U)[3], const R (&B)[3], const R (&b)[3], const R (&J)[3],
                          const R (&S)[3], R alpha, R omega_b) {
  const R V[3] = {U[0] - alpha * J[0], U[1] - alpha * J[1], U[2] - alpha * J[2]};
  R E[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) E[a][c] = V[a] * B[c] - B[a] * V[c];
  const R src = R(1) - R(0.5) * omega_b;
#pragma unroll
  for (int i = 0; i < ML::m; ++i) {
    const R W = R(ML::w(i));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R x = R(0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (ML::xi(i, a) == 1) x += E[a][c];
        else if (ML::xi(i, a) == -1) x -= E[a][c];
      }
      const R eq = W * (b[c] + R(4) * x);
      R& v = g[i * 3 + c];
      v = v - omega_b * (v - eq) + src * W * S[c];
    }
  }
}

// Deviation of the second-order equilibrium with the Maxwell stress from the rest state, without
// cancellation: f^mhd(0)_i - f_rest_i = w_i [d rho (1 + e_i) + e_i] + (w_i / 2 c_s^4)(M(B) - M(b0)) :
// (c c - c_s^2 I), e_i = 3 c.U + 9/2 (c.U)^2 - 3/2 |U|^2 (c_s^2 = 1/3).
template <typename FL, typename R>
FLAME_HD R eq2_deviation(int i, R drho, const R (&U)[3], R u2, R s, const R (&b)[3], const R (&b0)[3]) {
  const R cu = R(FL::c(i, 0)) * U[0] + R(FL::c(i, 1)) * U[1] + R(FL::c(i, 2)) * U[2];
  const R e = R(3) * cu + R(4.5) * cu * cu - R(1.5) * u2;
  const R w = R(FL::w(i));
  R v = w * (drho * (R(1) + e) + e);
  const R bc = R(FL::c(i, 0)) * b[0] + R(FL::c(i, 1)) * b[1] + R(FL::c(i, 2)) * b[2];
  const R b0c = R(FL::c(i, 0)) * b0[0] + R(FL::c(i, 1)) * b0[1] + R(FL::c(i, 2)) * b0[2];
  v += (w * R(4.5)) * (s * R(FL::speed2(i) - 1.0 / 3.0) - bc * (R(2) * b0c + bc));
  return v;
}

// Second-order force distribution along the force F: sum_a F_a w_i [(c_ia - U_a) / c_s^2 +
// (c_i . U) c_ia / c_s^4].
template <typename FL, typename R>
FLAME_HD R force2(int i, const R (&U)[3], const R (&F)[3]) {
  const R cu = R(FL::c(i, 0)) * U[0] + R(FL::c(i, 1)) * U[1] + R(FL::c(i, 2)) * U[2];
  R v = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) v += F[a] * (R(3) * (R(FL::c(i, a)) - U[a]) + R(9) * cu * R(FL::c(i, a)));
  return R(FL::w(i)) * v;
}

// D3Q19 BGK collision in deviations: f* = f0 + (1 - w)(f - f0) + (1 - w/2) force2.
template <typename FL, typename R>
FLAME_HD void collide_fluid_bgk2(R (&f)[FL::q], R drho, const R (&U)[3], const R (&b)[3], const R (&b0)[3],
                                 const R (&F)[3], R omega) {
  const R u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  const R s = b0[0] * b[0] + b0[1] * b[1] + b0[2] * b[2] + R(0.5) * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  const R om1 = R(1) - omega;
  const R fk = R(1) - R(0.5) * omega;
#pragma unroll
  for (int i = 0; i < FL::q; ++i) {
    const R eq = eq2_deviation<FL>(i, drho, U, u2, s, b, b0);
    f[i] = eq + om1 * (f[i] - eq) + fk * force2<FL>(i, U, F);
  }
}

// Fluid collision on the set FL: D3Q27 keeps the paper's central-moment operator (or its BGK
// limit); D3Q19 runs the BGK operator above.
template <typename FL, bool BGK, typename R>
FLAME_HD void collide_fluid_set(R (&f)[FL::q], R drho, const R (&U)[3], const R (&b)[3], const R (&b0)[3],
                                const R (&F)[3], R omega) {
  if constexpr (FL::q == 27) {
    const FluidMoments<R> m = fluid_moments(f);
    if constexpr (BGK)
      collide_fluid_bgk(f, m, U, b, b0, F, omega);
    else
      collide_fluid<R, false>(f, m, R(1) + m.drho, U, b, b0, F, omega);
  } else {
    collide_fluid_bgk2<FL>(f, drho, U, b, b0, F, omega);
  }
}

// The whole collision of one node on deviations (moments, J from the magnetic moments, fluid and
// magnetic collisions), in place: the arithmetic of the variant step between its loads and stores.
template <typename FL, typename ML, bool BGK, bool EMHD, typename R>
FLAME_HD void variant_node(R (&f)[FL::q], R (&g)[ML::m * 3], const R (&F)[3], const R (&Sb)[3],
                           const PhysConst<R>& k) {
  R drho = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < FL::q; ++i) {
    drho += f[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (FL::c(i, c) == 1) j[c] += f[i];
      else if (FL::c(i, c) == -1) j[c] -= f[i];
    }
  }
  const R inv_rho = R(1) / (R(1) + drho);
  const R U[3] = {(j[0] + R(0.5) * F[0]) * inv_rho, (j[1] + R(0.5) * F[1]) * inv_rho, (j[2] + R(0.5) * F[2]) * inv_rho};
  R b[3], lam[3][3];
  mag_moments<ML>(g, b, lam);
#pragma unroll
  for (int c = 0; c < 3; ++c) b[c] += R(0.5) * Sb[c];
  const R b0[3] = {k.b0[0], k.b0[1], k.b0[2]};
  const R B[3] = {b0[0] + b[0], b0[1] + b[1], b0[2] + b[2]};
  const R zero[3] = {R(0), R(0), R(0)};
  const R(&Um)[3] = EMHD ? zero : U;
  R J[3];
  current_from_moments(lam, Um, B, k.alpha, k.omega_b, J);
  collide_fluid_set<FL, BGK>(f, drho, U, b, b0, F, k.omega);
  collide_mag<ML>(g, Um, B, b, J, Sb, k.alpha, k.omega_b);
}

}  // namespace lattice
}  // namespace flame
