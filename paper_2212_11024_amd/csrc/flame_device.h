// Device-side lattice tables, storage encodings and per-node arithmetic of the coupled
// Hall-MHD lattice-Boltzmann step (paper Sec. 3.1-3.2, App. A-B).
//
// Populations are carried as deviations from the rest state of the run,
//   df_i = f_i - f_rest_i,  f_rest = f^mhd(0)(1, 0, b0);   dg_ia = g_ia - W_i b0_a,
// so that FP32/FP16 storage keeps its precision for the small departures that carry the
// physics. All per-node arithmetic below is written in terms of these deviations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-node arithmetic is host-and-device so the same code can be exercised on the CPU.
#define FLAME_HD __host__ __device__ __forceinline__

namespace flame {

// ------------------------------------------------------------------ lattice tables
// D3Q27 velocities in the order of the paper's App. A listing.
__host__ __device__ constexpr int cq(int i, int a) {
  constexpr int8_t t[27][3] = {
      {0, 0, 0},   {-1, 0, 0},  {0, -1, 0},  {0, 0, -1}, {-1, -1, 0}, {-1, 1, 0},  {-1, 0, -1},
      {-1, 0, 1},  {0, -1, -1}, {0, -1, 1},  {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
      {1, 0, 0},   {0, 1, 0},   {0, 0, 1},   {1, 1, 0},  {1, -1, 0},  {1, 0, 1},   {1, 0, -1},
      {0, 1, 1},   {0, 1, -1},  {1, 1, 1},   {1, 1, -1}, {1, -1, 1},  {1, -1, -1}};
  return t[i][a];
}
// In the App. A listing the opposite of direction i (1 <= i <= 13) is i + 13.
__host__ __device__ constexpr int oppq(int i) { return i == 0 ? 0 : (i <= 13 ? i + 13 : i - 13); }
// Index of the D3Q27 direction (x, y, z) in the App. A order.
__host__ __device__ constexpr int qindex(int x, int y, int z) {
  int k = 0;
  for (int i = 0; i < 27; ++i)
    if (cq(i, 0) == x && cq(i, 1) == y && cq(i, 2) == z) k = i;
  return k;
}
__host__ __device__ constexpr int speed2q(int i) {
  return cq(i, 0) * cq(i, 0) + cq(i, 1) * cq(i, 1) + cq(i, 2) * cq(i, 2);
}
// Weights by speed class (Sec. 3.1): 8/27, 2/27, 1/54, 1/216.
__host__ __device__ constexpr double wq(int i) {
  return speed2q(i) == 0 ? 8.0 / 27.0
       : speed2q(i) == 1 ? 2.0 / 27.0
       : speed2q(i) == 2 ? 1.0 / 54.0
                          : 1.0 / 216.0;
}
// D3Q7: rest, -x, -y, -z, +x, +y, +z. Weights 1/4 (rest), 1/8 (faces); C^2 = 1/4.
__host__ __device__ constexpr int xim(int i, int a) {
  return i == 0 ? 0 : (i <= 3 ? (a == i - 1 ? -1 : 0) : (a == i - 4 ? 1 : 0));
}
__host__ __device__ constexpr int oppm(int i) { return i == 0 ? 0 : (i <= 3 ? i + 3 : i - 3); }
__host__ __device__ constexpr double wm(int i) { return i == 0 ? 0.25 : 0.125; }

constexpr int kQ = 27;
constexpr int kM = 21;   // 7 directions x 3 components, index i * 3 + component

// ------------------------------------------------------------------ storage encodings
// Power-of-two scales applied to stored deviations (exact in every format); only FP16
// needs them, to keep deviations of magnitude ~ w_i |u| clear of the subnormal range.
template <typename S>
struct Enc;

template <>
struct Enc<double> {
  using R = double;
  static __host__ __device__ constexpr double fscale(int) { return 1.0; }
  static __host__ __device__ constexpr double mscale(int) { return 1.0; }
  static __device__ __forceinline__ double dec(double v, double) { return v; }
  static __device__ __forceinline__ double enc(double v, double) { return v; }
};

template <>
struct Enc<float> {
  using R = float;
  static __host__ __device__ constexpr double fscale(int) { return 1.0; }
  static __host__ __device__ constexpr double mscale(int) { return 1.0; }
  static __device__ __forceinline__ float dec(float v, float) { return v; }
  static __device__ __forceinline__ float enc(float v, float) { return v; }
};

template <>
struct Enc<_Float16> {
  using R = float;
  static __host__ __device__ constexpr double fscale(int i) {
    return speed2q(i) == 0 ? 4.0 : speed2q(i) == 1 ? 16.0 : speed2q(i) == 2 ? 64.0 : 256.0;
  }
  static __host__ __device__ constexpr double mscale(int i) { return i == 0 ? 4.0 : 8.0; }
  static __device__ __forceinline__ float dec(_Float16 v, float inv_scale) {
    return static_cast<float>(v) * inv_scale;
  }
  static __device__ __forceinline__ _Float16 enc(float v, float scale) {
    return static_cast<_Float16>(v * scale);
  }
};

// ------------------------------------------------------------------ run constants
template <typename R>
struct PhysConst {
  R omega;       // fluid relaxation rate, 1/omega = 3 nu + 1/2
  R omega_b;     // magnetic relaxation rate, 1/omega_B = 4 eta + 1/2
  R alpha;       // Hall coefficient alpha_H (= d_i in cells)
  R b0[3];       // background field
};

// ------------------------------------------------------------------ per-node arithmetic
// Fluid moments of the deviations: d rho = sum df, j = sum df c, S2 = sum df c c.
template <typename R>
struct FluidMoments {
  R drho, jx, jy, jz, sxx, syy, szz, sxy, sxz, syz;
};

template <typename R>
FLAME_HD FluidMoments<R> fluid_moments(const R (&f)[kQ]) {
  FluidMoments<R> m{};
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const R v = f[i];
    m.drho += v;
    if (cq(i, 0) == 1) m.jx += v; else if (cq(i, 0) == -1) m.jx -= v;
    if (cq(i, 1) == 1) m.jy += v; else if (cq(i, 1) == -1) m.jy -= v;
    if (cq(i, 2) == 1) m.jz += v; else if (cq(i, 2) == -1) m.jz -= v;
    if (cq(i, 0) != 0) m.sxx += v;
    if (cq(i, 1) != 0) m.syy += v;
    if (cq(i, 2) != 0) m.szz += v;
    if (cq(i, 0) * cq(i, 1) == 1) m.sxy += v; else if (cq(i, 0) * cq(i, 1) == -1) m.sxy -= v;
    if (cq(i, 0) * cq(i, 2) == 1) m.sxz += v; else if (cq(i, 0) * cq(i, 2) == -1) m.sxz -= v;
    if (cq(i, 1) * cq(i, 2) == 1) m.syz += v; else if (cq(i, 1) * cq(i, 2) == -1) m.syz -= v;
  }
  return m;
}

// Field fluctuation b = sum dg (the rest part sums to b0) and Lambda_ab = sum_i xi_ia g_ib,
// which for D3Q7 is the difference of the +a and -a populations (the rest part cancels).
template <typename R>
FLAME_HD void magnetic_moments(const R (&g)[kM], R (&b)[3], R (&lam)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R s = g[a];
#pragma unroll
    for (int i = 1; i < 7; ++i) s += g[i * 3 + a];
    b[a] = s;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) lam[a][c] = g[(4 + a) * 3 + c] - g[(1 + a) * 3 + c];
}

// Field fluctuation component c of a node from its magnetic populations, with the source
// half-shift; one fixed summation order everywhere so a node's b is bitwise the same
// whichever thread computes it.
template <typename R>
FLAME_HD R b_component(const R (&g)[kM], int c, R half_src) {
  R s = g[c];
#pragma unroll
  for (int i = 1; i < 7; ++i) s += g[i * 3 + c];
  return s + half_src;
}

// J from the magnetic first moment (Sec. 3.2): (I + 2 alpha w_B / C^2 M(B)) J = -(w_B/C^2) J0,
// M(B) J = J x B, J0 = eps:Lambda - 2 U x B. Written as J + k (J x B) = r, whose solution is
// J = (r - k r x B + k^2 (r . B) B) / (1 + k^2 |B|^2), with k = 8 alpha w_B and r = -4 w_B J0.
template <typename R>
FLAME_HD void current_from_moments(const R (&lam)[3][3], const R (&U)[3],
                                                     const R (&B)[3], R alpha, R omega_b,
                                                     R (&J)[3]) {
  const R j0x = lam[1][2] - lam[2][1] - R(2) * (U[1] * B[2] - U[2] * B[1]);
  const R j0y = lam[2][0] - lam[0][2] - R(2) * (U[2] * B[0] - U[0] * B[2]);
  const R j0z = lam[0][1] - lam[1][0] - R(2) * (U[0] * B[1] - U[1] * B[0]);
  const R s = R(-4) * omega_b;
  const R rx = s * j0x, ry = s * j0y, rz = s * j0z;
  const R k = R(8) * alpha * omega_b;
  const R rbx = ry * B[2] - rz * B[1], rby = rz * B[0] - rx * B[2], rbz = rx * B[1] - ry * B[0];
  const R rdb = rx * B[0] + ry * B[1] + rz * B[2];
  const R k2 = k * k;
  const R inv = R(1) / (R(1) + k2 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]));
  J[0] = (rx - k * rbx + k2 * rdb * B[0]) * inv;
  J[1] = (ry - k * rby + k2 * rdb * B[1]) * inv;
  J[2] = (rz - k * rbz + k2 * rdb * B[2]) * inv;
}

// 1-D factors on c in {-1, 0, +1} (index c + 1):
//  e(c) = phi(c; u) / w1(c) - 1, phi the D1Q3 equilibrium (its 3-D product is the
//        sixth-order Hermite f^(0) of App. A): e(0) = -3u^2/2, e(+-1) = 3u^2 +- 3u;
//  h_p(c): central moments about u equal to delta_{p,q} for q = 0, 1, 2.
template <typename R>
struct Axis {
  R e[3], h0[3], h1[3], h2[3];
  FLAME_HD explicit Axis(R u) {
    const R u2 = u * u;
    e[0] = R(3) * (u2 - u); e[1] = R(-1.5) * u2; e[2] = R(3) * (u2 + u);
    h0[0] = R(0.5) * (u2 - u); h0[1] = R(1) - u2; h0[2] = R(0.5) * (u2 + u);
    h1[0] = u - R(0.5); h1[1] = R(-2) * u; h1[2] = u + R(0.5);
    h2[0] = R(0.5); h2[1] = R(-1); h2[2] = R(0.5);
  }
};

// Post-collision fluid deviations, in place (Sec. 3.1.2 with S = diag[1,1,1,1,w x5,1 x18]).
// Because every moment except the five deviatoric second-order ones relaxes to equilibrium
// with rate 1, the back-transform of the collided central moments is
//   f*_i = f^mhd(0)_i + (1 - w) sum_ab P_ab H^ab_i + sum_a (F_a/2) H^a_i,
// with P the deviatoric second central moment of f - f^mhd(0), H^ab = h..(c_x) h..(c_y) h..(c_z)
// the distributions with a single unit central moment, and F the body force (its half enters
// the velocity, the collision sets the first central moment to +F/2).
// In deviations: f^mhd(0)_i - f_rest_i = w_i [d rho E_i + (E_i - 1)] + (w_i / 2 c_s^4)
// (M(B) - M(b0)) : (c c - c_s^2 I), E_i = prod_a (1 + e_a), M(B) = |B|^2/2 I - B B.
//
// Grouped selects the order in which the 27 directions are formed: false, one direction at a time
// in the App. A order; true, by (c_x, c_y) columns sharing their x/y factors, which shortens live
// ranges (fewer registers). Both give the same values; the grouped order pays where the step is
// arithmetic-bound (FP16 storage) and costs write combining in the odd AA step where it is not.
template <typename R, bool Grouped = false>
FLAME_HD void collide_fluid(R (&f)[kQ], const FluidMoments<R>& m, R rho,
                                              const R (&U)[3], const R (&b)[3], const R (&b0)[3],
                                              const R (&F)[3], R omega) {
  // deviatoric K = S2 - rho U U + (U F + F U)/2 + (B B - b0 b0); B B - b0 b0 = b0 b + b b0 + b b
  const R kxx = m.sxx - rho * U[0] * U[0] + U[0] * F[0] + b[0] * (R(2) * b0[0] + b[0]);
  const R kyy = m.syy - rho * U[1] * U[1] + U[1] * F[1] + b[1] * (R(2) * b0[1] + b[1]);
  const R kzz = m.szz - rho * U[2] * U[2] + U[2] * F[2] + b[2] * (R(2) * b0[2] + b[2]);
  const R om1 = R(1) - omega;
  const R tr = (kxx + kyy + kzz) * R(1.0 / 3.0);
  const R qxx = om1 * (kxx - tr), qyy = om1 * (kyy - tr), qzz = om1 * (kzz - tr);
  const R qxy = om1 * (m.sxy - rho * U[0] * U[1] + R(0.5) * (U[0] * F[1] + F[0] * U[1])
                       + b0[0] * b[1] + b[0] * b0[1] + b[0] * b[1]);
  const R qxz = om1 * (m.sxz - rho * U[0] * U[2] + R(0.5) * (U[0] * F[2] + F[0] * U[2])
                       + b0[0] * b[2] + b[0] * b0[2] + b[0] * b[2]);
  const R qyz = om1 * (m.syz - rho * U[1] * U[2] + R(0.5) * (U[1] * F[2] + F[1] * U[2])
                       + b0[1] * b[2] + b[1] * b0[2] + b[1] * b[2]);
  const R fhx = R(0.5) * F[0], fhy = R(0.5) * F[1], fhz = R(0.5) * F[2];
  // Maxwell-stress change: (M(B) - M(b0)) : (cc - I/3) = s (|c|^2 - 1/3) - (b.c)(2 b0.c + b.c)
  const R s = b0[0] * b[0] + b0[1] * b[1] + b0[2] * b[2]
            + R(0.5) * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  const Axis<R> ax(U[0]), ay(U[1]), az(U[2]);
  const R drho = m.drho;
  // each direction: equilibrium deviation w_i [d rho E_i + (E_i - 1)], the Maxwell-stress change,
  // and the collided second moments and force through the h-factors
  if constexpr (Grouped) {
#pragma unroll
    for (int X = 0; X < 3; ++X) {
#pragma unroll
      for (int Y = 0; Y < 3; ++Y) {
        const R h0x = ax.h0[X], h0y = ay.h0[Y], h1x = ax.h1[X], h1y = ay.h1[Y], h2x = ax.h2[X], h2y = ay.h2[Y];
        const R p00 = h0x * h0y;
        const R A0 = h2x * h0y * qxx + h0x * h2y * qyy + h1x * h1y * qxy + h1x * h0y * fhx + h0x * h1y * fhy;
        const R A1 = h1x * h0y * qxz + h0x * h1y * qyz + p00 * fhz;
        const R A2 = p00 * qzz;
        const R ex = ax.e[X], ey = ay.e[Y];
#pragma unroll
        for (int Z = 0; Z < 3; ++Z) {
          const int i = qindex(X - 1, Y - 1, Z - 1);
          const R ez = az.e[Z];
          const R em1 = ex + (R(1) + ex) * (ey + (R(1) + ey) * ez);   // E_i - 1 without cancellation
          const R w = R(wq(i));
          R v = w * (drho * (R(1) + em1) + em1);
          const R bc = R(cq(i, 0)) * b[0] + R(cq(i, 1)) * b[1] + R(cq(i, 2)) * b[2];
          const R b0c = R(cq(i, 0)) * b0[0] + R(cq(i, 1)) * b0[1] + R(cq(i, 2)) * b0[2];
          v += (w * R(4.5)) * (s * R(speed2q(i) - 1.0 / 3.0) - bc * (R(2) * b0c + bc));
          v += az.h0[Z] * A0 + az.h1[Z] * A1 + az.h2[Z] * A2;
          f[i] = v;
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int x = cq(i, 0) + 1, y = cq(i, 1) + 1, z = cq(i, 2) + 1;
      const R ex = ax.e[x], ey = ay.e[y], ez = az.e[z];
      const R em1 = ex + (R(1) + ex) * (ey + (R(1) + ey) * ez);   // E_i - 1 without cancellation
      const R w = R(wq(i));
      R v = w * (drho * (R(1) + em1) + em1);
      const R bc = R(cq(i, 0)) * b[0] + R(cq(i, 1)) * b[1] + R(cq(i, 2)) * b[2];
      const R b0c = R(cq(i, 0)) * b0[0] + R(cq(i, 1)) * b0[1] + R(cq(i, 2)) * b0[2];
      v += (w * R(4.5)) * (s * R(speed2q(i) - 1.0 / 3.0) - bc * (R(2) * b0c + bc));
      const R h0x = ax.h0[x], h0y = ay.h0[y], h0z = az.h0[z];
      const R h1x = ax.h1[x], h1y = ay.h1[y], h1z = az.h1[z];
      const R h2x = ax.h2[x], h2y = ay.h2[y], h2z = az.h2[z];
      v += h0z * (h2x * h0y * qxx + h0x * h2y * qyy + h1x * h1y * qxy + h1x * h0y * fhx + h0x * h1y * fhy)
         + h1z * (h1x * h0y * qxz + h0x * h1y * qyz + h0x * h0y * fhz)
         + h2z * (h0x * h0y * qzz);
      f[i] = v;
    }
  }
}

// Post-collision magnetic deviations, in place (eq. MHD_LBscheme with the Hall equilibrium
// gHall_eq): g* = g - w_B (g - g^Hall(0)) + (1 - w_B/2) W_i S. With V = U - alpha J and
// E_ac = V_a B_c - B_a V_c, g^Hall(0)_{+-a, c} = W (B_c +- 4 E_ac), g^Hall(0)_{0, c} = W_0 B_c.
template <typename R>
FLAME_HD void collide_magnetic(R (&g)[kM], const R (&U)[3], const R (&B)[3],
                                                 const R (&b)[3], const R (&J)[3],
                                                 const R (&S)[3], R alpha, R omega_b) {
  const R V[3] = {U[0] - alpha * J[0], U[1] - alpha * J[1], U[2] - alpha * J[2]};
  const R src = R(1) - R(0.5) * omega_b;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R eq0 = R(0.25) * b[c];
    g[c] = g[c] - omega_b * (g[c] - eq0) + src * R(0.25) * S[c];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R E = (a == c) ? R(0) : (V[a] * B[c] - B[a] * V[c]);
      const R eqp = R(0.125) * (b[c] + R(4) * E);
      const R eqm = R(0.125) * (b[c] - R(4) * E);
      const int ip = (4 + a) * 3 + c, im = (1 + a) * 3 + c;
      g[ip] = g[ip] - omega_b * (g[ip] - eqp) + src * R(0.125) * S[c];
      g[im] = g[im] - omega_b * (g[im] - eqm) + src * R(0.125) * S[c];
    }
  }
}

// ------------------------------------------------------------------ per-node reverse pass
// Derivatives of the 1-D factors of Axis with respect to u (h2 is constant).
// BGK variant of the fluid collision, in place on deviations: the central-moment step with every
// rate equal to w (Sec. 3.1.2; the standard operator of Sec. 3.1.1),
//   f*_i = f^mhd(0)_i + (1 - w)(f_i - f^mhd(0)_i) + (1 - w/2) sum_a F_a H^a_i.
// The force term ends the first central moments at +F/2 as in collide_fluid: before the
// collision those of f - f^mhd(0) are -F/2 (U carries F/2), and (1 - w) of them survive.
// f^mhd(0) - f_rest is the same equilibrium deviation as in collide_fluid.
template <typename R>
FLAME_HD void collide_fluid_bgk(R (&f)[kQ], const FluidMoments<R>& m, const R (&U)[3], const R (&b)[3],
                                const R (&b0)[3], const R (&F)[3], R omega) {
  const R s = b0[0] * b[0] + b0[1] * b[1] + b0[2] * b[2] + R(0.5) * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  const Axis<R> ax(U[0]), ay(U[1]), az(U[2]);
  const R drho = m.drho;
  const R om1 = R(1) - omega;
  const R fk = R(1) - R(0.5) * omega;
  const R fx = fk * F[0], fy = fk * F[1], fz = fk * F[2];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int x = cq(i, 0) + 1, y = cq(i, 1) + 1, z = cq(i, 2) + 1;
    const R ex = ax.e[x], ey = ay.e[y], ez = az.e[z];
    const R em1 = ex + (R(1) + ex) * (ey + (R(1) + ey) * ez);   // E_i - 1 without cancellation
    const R w = R(wq(i));
    R eq = w * (drho * (R(1) + em1) + em1);
    const R bc = R(cq(i, 0)) * b[0] + R(cq(i, 1)) * b[1] + R(cq(i, 2)) * b[2];
    const R b0c = R(cq(i, 0)) * b0[0] + R(cq(i, 1)) * b0[1] + R(cq(i, 2)) * b0[2];
    eq += (w * R(4.5)) * (s * R(speed2q(i) - 1.0 / 3.0) - bc * (R(2) * b0c + bc));
    const R force = ax.h1[x] * ay.h0[y] * az.h0[z] * fx + ax.h0[x] * ay.h1[y] * az.h0[z] * fy
                  + ax.h0[x] * ay.h0[y] * az.h1[z] * fz;
    f[i] = eq + om1 * (f[i] - eq) + force;
  }
}

template <typename R>
struct AxisD {
  R de[3], dh0[3], dh1[3];
  FLAME_HD explicit AxisD(R u) {
    de[0] = R(6) * u - R(3); de[1] = R(-3) * u; de[2] = R(6) * u + R(3);
    dh0[0] = u - R(0.5); dh0[1] = R(-2) * u; dh0[2] = u + R(0.5);
    dh1[0] = R(1); dh1[1] = R(-2); dh1[2] = R(1);
  }
};

// Vector-Jacobian product of one node's collision (the adjoint of collide_fluid +
// collide_magnetic with the moments and, on the moment route, J recomputed from the node's
// pre-collision deviations f, g). Given mf, mg = d loss / d(post-collision deviations), returns
// lf, lg = d loss / d(pre-collision deviations) through this node's collision, and lJ =
// d loss / dJ (stencil route: J is an input computed from neighbouring fields, Jst; on the moment
// route lJ is folded into lf, lg and returned as zero). F, S: forcing at the node.
// Forward quantities of one node that the reverse pass needs (recomputed from the pre-collision
// state; J from the moments on the moment route, else the J the forward step used).
template <typename R>
struct VjpState {
  FluidMoments<R> m;
  R rho, inv_rho, U[3], b[3], B[3], J[3], V[3], lam[3][3];
};

template <typename R, bool MOMENT>
FLAME_HD VjpState<R> vjp_forward(const R (&f)[kQ], const R (&g)[kM], const R (&F)[3], const R (&S)[3],
                                 const R (&Jst)[3], const PhysConst<R>& k) {
  VjpState<R> st;
  st.m = fluid_moments(f);
  st.rho = R(1) + st.m.drho;
  st.inv_rho = R(1) / st.rho;
  st.U[0] = (st.m.jx + R(0.5) * F[0]) * st.inv_rho;
  st.U[1] = (st.m.jy + R(0.5) * F[1]) * st.inv_rho;
  st.U[2] = (st.m.jz + R(0.5) * F[2]) * st.inv_rho;
  magnetic_moments(g, st.b, st.lam);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    st.b[c] += R(0.5) * S[c];
    st.B[c] = k.b0[c] + st.b[c];
  }
  if (MOMENT) current_from_moments(st.lam, st.U, st.B, k.alpha, k.omega_b, st.J);
  else { st.J[0] = Jst[0]; st.J[1] = Jst[1]; st.J[2] = Jst[2]; }
#pragma unroll
  for (int c = 0; c < 3; ++c) st.V[c] = st.U[c] - k.alpha * st.J[c];
  return st;
}

// The reverse pass proper: lf, lg, lJ from the adjoints mf, mg of the post-collision populations
// at the forward quantities st. It reads neither the pre-collision populations nor S, so a kernel
// can drop those before it gathers mf and mg.
template <typename R, bool MOMENT>
FLAME_HD void vjp_reverse(const VjpState<R>& st, const R (&F)[3], const PhysConst<R>& k, const R (&mf)[kQ],
                          const R (&mg)[kM], R (&lf)[kQ], R (&lg)[kM], R (&lJ)[3]) {
  const FluidMoments<R>& m = st.m;
  const R rho = st.rho, inv_rho = st.inv_rho;
  const R(&U)[3] = st.U;
  const R(&b)[3] = st.b;
  const R(&B)[3] = st.B;
  const R(&J)[3] = st.J;
  const R(&V)[3] = st.V;
  const R(&lam)[3][3] = st.lam;
  const R b0[3] = {k.b0[0], k.b0[1], k.b0[2]};
  R lU[3] = {R(0), R(0), R(0)}, lb[3] = {R(0), R(0), R(0)}, lB[3] = {R(0), R(0), R(0)};
  R lrho = R(0);
  R llam[3][3] = {};

  // ---- magnetic: g* = (1 - w_B) g + w_B g^Hall(0)(b, E) + source
  {
    const R ob = k.omega_b;
#pragma unroll
    for (int q = 0; q < kM; ++q) lg[q] = (R(1) - ob) * mg[q];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R acc = R(0.25) * ob * mg[c];
#pragma unroll
      for (int a = 0; a < 3; ++a) acc += R(0.125) * ob * (mg[(4 + a) * 3 + c] + mg[(1 + a) * 3 + c]);
      lb[c] += acc;
    }
    R lV[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (a == c) continue;
        // g^Hall(0)_{+-a, c} = W (b_c +- 4 E_ac), W = 1/8, E_ac = V_a B_c - B_a V_c
        const R lE = R(0.5) * ob * (mg[(4 + a) * 3 + c] - mg[(1 + a) * 3 + c]);
        lV[a] += lE * B[c];
        lB[c] += lE * V[a];
        lB[a] -= lE * V[c];
        lV[c] -= lE * B[a];
      }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lU[a] += lV[a];
      lJ[a] = -k.alpha * lV[a];
    }
  }

  // ---- current from the moments: J = N / D, N = r - kk r x B + kk^2 (r.B) B, D = 1 + kk^2 |B|^2,
  //      r = -4 w_B J0, J0 = A(Lambda) - 2 U x B
  if (MOMENT) {
    const R kk = R(8) * k.alpha * k.omega_b;
    const R kk2 = kk * kk;
    const R D = R(1) + kk2 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const R j0[3] = {lam[1][2] - lam[2][1] - R(2) * (U[1] * B[2] - U[2] * B[1]),
                     lam[2][0] - lam[0][2] - R(2) * (U[2] * B[0] - U[0] * B[2]),
                     lam[0][1] - lam[1][0] - R(2) * (U[0] * B[1] - U[1] * B[0])};
    const R r[3] = {R(-4) * k.omega_b * j0[0], R(-4) * k.omega_b * j0[1], R(-4) * k.omega_b * j0[2]};
    const R lN[3] = {lJ[0] / D, lJ[1] / D, lJ[2] / D};
    const R lD = -(lJ[0] * J[0] + lJ[1] * J[1] + lJ[2] * J[2]) / D;
    const R BlN = B[0] * lN[0] + B[1] * lN[1] + B[2] * lN[2];
    const R rB = r[0] * B[0] + r[1] * B[1] + r[2] * B[2];
    // d/dr:  lN - kk (B x lN) + kk^2 (B.lN) B
    const R Bxl[3] = {B[1] * lN[2] - B[2] * lN[1], B[2] * lN[0] - B[0] * lN[2], B[0] * lN[1] - B[1] * lN[0]};
    R lr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) lr[a] = lN[a] - kk * Bxl[a] + kk2 * BlN * B[a];
    // d/dB: -kk (lN x r) + kk^2 ((B.lN) r + (r.B) lN) + 2 kk^2 lD B
    const R lxr[3] = {lN[1] * r[2] - lN[2] * r[1], lN[2] * r[0] - lN[0] * r[2], lN[0] * r[1] - lN[1] * r[0]};
#pragma unroll
    for (int a = 0; a < 3; ++a) lB[a] += -kk * lxr[a] + kk2 * (BlN * r[a] + rB * lN[a]) + R(2) * kk2 * lD * B[a];
    const R lj0[3] = {R(-4) * k.omega_b * lr[0], R(-4) * k.omega_b * lr[1], R(-4) * k.omega_b * lr[2]};
    // J0 = A - 2 U x B: d/dU = -2 (B x lj0), d/dB = -2 (lj0 x U)
    const R Bxj[3] = {B[1] * lj0[2] - B[2] * lj0[1], B[2] * lj0[0] - B[0] * lj0[2], B[0] * lj0[1] - B[1] * lj0[0]};
    const R jxU[3] = {lj0[1] * U[2] - lj0[2] * U[1], lj0[2] * U[0] - lj0[0] * U[2], lj0[0] * U[1] - lj0[1] * U[0]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lU[a] += R(-2) * Bxj[a];
      lB[a] += R(-2) * jxU[a];
    }
    llam[1][2] += lj0[0]; llam[2][1] -= lj0[0];
    llam[2][0] += lj0[1]; llam[0][2] -= lj0[1];
    llam[0][1] += lj0[2]; llam[1][0] -= lj0[2];
    lJ[0] = lJ[1] = lJ[2] = R(0);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) lb[a] += lB[a];

  // ---- fluid: f*_i = w_i (rho E_i - 1) + Maxwell_i(b) + sum_p Q_p H^p_i(U) + sum_a (F_a/2) H^a_i(U)
  {
    const R om1 = R(1) - k.omega;
    const R kxx = m.sxx - rho * U[0] * U[0] + U[0] * F[0] + b[0] * (R(2) * b0[0] + b[0]);
    const R kyy = m.syy - rho * U[1] * U[1] + U[1] * F[1] + b[1] * (R(2) * b0[1] + b[1]);
    const R kzz = m.szz - rho * U[2] * U[2] + U[2] * F[2] + b[2] * (R(2) * b0[2] + b[2]);
    const R tr = (kxx + kyy + kzz) * R(1.0 / 3.0);
    const R qxx = om1 * (kxx - tr), qyy = om1 * (kyy - tr), qzz = om1 * (kzz - tr);
    const R qxy = om1 * (m.sxy - rho * U[0] * U[1] + R(0.5) * (U[0] * F[1] + F[0] * U[1])
                         + b0[0] * b[1] + b[0] * b0[1] + b[0] * b[1]);
    const R qxz = om1 * (m.sxz - rho * U[0] * U[2] + R(0.5) * (U[0] * F[2] + F[0] * U[2])
                         + b0[0] * b[2] + b[0] * b0[2] + b[0] * b[2]);
    const R qyz = om1 * (m.syz - rho * U[1] * U[2] + R(0.5) * (U[1] * F[2] + F[1] * U[2])
                         + b0[1] * b[2] + b[1] * b0[2] + b[1] * b[2]);
    const R fhx = R(0.5) * F[0], fhy = R(0.5) * F[1], fhz = R(0.5) * F[2];
    const Axis<R> ax(U[0]), ay(U[1]), az(U[2]);
    const AxisD<R> dx(U[0]), dy(U[1]), dz(U[2]);
    R lqxx = R(0), lqyy = R(0), lqzz = R(0), lqxy = R(0), lqxz = R(0), lqyz = R(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int x = cq(i, 0) + 1, y = cq(i, 1) + 1, z = cq(i, 2) + 1;
      const R mu = mf[i];
      const R w = R(wq(i));
      const R ex = R(1) + ax.e[x], ey = R(1) + ay.e[y], ez = R(1) + az.e[z];
      lrho += mu * w * ex * ey * ez;
      const R wr = mu * w * rho;
      lU[0] += wr * dx.de[x] * ey * ez;
      lU[1] += wr * ex * dy.de[y] * ez;
      lU[2] += wr * ex * ey * dz.de[z];
      const R Bc = R(cq(i, 0)) * B[0] + R(cq(i, 1)) * B[1] + R(cq(i, 2)) * B[2];
      const R wm45 = mu * w * R(4.5);
      const R c2 = R(speed2q(i) - 1.0 / 3.0);
      lb[0] += wm45 * (B[0] * c2 - R(2 * cq(i, 0)) * Bc);
      lb[1] += wm45 * (B[1] * c2 - R(2 * cq(i, 1)) * Bc);
      lb[2] += wm45 * (B[2] * c2 - R(2 * cq(i, 2)) * Bc);
      const R h0x = ax.h0[x], h0y = ay.h0[y], h0z = az.h0[z];
      const R h1x = ax.h1[x], h1y = ay.h1[y], h1z = az.h1[z];
      const R h2x = ax.h2[x], h2y = ay.h2[y], h2z = az.h2[z];
      const R d0x = dx.dh0[x], d0y = dy.dh0[y], d0z = dz.dh0[z];
      const R d1x = dx.dh1[x], d1y = dy.dh1[y], d1z = dz.dh1[z];
      lqxx += mu * h2x * h0y * h0z;
      lqyy += mu * h0x * h2y * h0z;
      lqzz += mu * h0x * h0y * h2z;
      lqxy += mu * h1x * h1y * h0z;
      lqxz += mu * h1x * h0y * h1z;
      lqyz += mu * h0x * h1y * h1z;
      lU[0] += mu * (qyy * d0x * h2y * h0z + qzz * d0x * h0y * h2z + qxy * d1x * h1y * h0z + qxz * d1x * h0y * h1z
                     + qyz * d0x * h1y * h1z + fhx * d1x * h0y * h0z + fhy * d0x * h1y * h0z + fhz * d0x * h0y * h1z);
      lU[1] += mu * (qxx * h2x * d0y * h0z + qzz * h0x * d0y * h2z + qxy * h1x * d1y * h0z + qxz * h1x * d0y * h1z
                     + qyz * h0x * d1y * h1z + fhx * h1x * d0y * h0z + fhy * h0x * d1y * h0z + fhz * h0x * d0y * h1z);
      lU[2] += mu * (qxx * h2x * h0y * d0z + qyy * h0x * h2y * d0z + qxy * h1x * h1y * d0z + qxz * h1x * h0y * d1z
                     + qyz * h0x * h1y * d1z + fhx * h1x * h0y * d0z + fhy * h0x * h1y * d0z + fhz * h0x * h0y * d1z);
    }
    // Q = (1 - w) (K - tr K / 3 I): the deviatoric projection is self-adjoint
    const R ltr = (lqxx + lqyy + lqzz) * R(1.0 / 3.0);
    const R lk[3] = {om1 * (lqxx - ltr), om1 * (lqyy - ltr), om1 * (lqzz - ltr)};
    const R lkxy = om1 * lqxy, lkxz = om1 * lqxz, lkyz = om1 * lqyz;
    R ls2[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ls2[a] = lk[a];
      lrho -= lk[a] * U[a] * U[a];
      lU[a] += lk[a] * (R(-2) * rho * U[a] + F[a]);
      lb[a] += lk[a] * R(2) * B[a];
    }
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    const R lko[3] = {lkxy, lkxz, lkyz};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int a = pa[p], c = pb[p];
      ls2[3 + p] = lko[p];
      lrho -= lko[p] * U[a] * U[c];
      lU[a] += lko[p] * (-rho * U[c] + R(0.5) * F[c]);
      lU[c] += lko[p] * (-rho * U[a] + R(0.5) * F[a]);
      lb[a] += lko[p] * B[c];
      lb[c] += lko[p] * B[a];
    }
    // U = (j + F/2) / rho
    const R lj[3] = {lU[0] * inv_rho, lU[1] * inv_rho, lU[2] * inv_rho};
    lrho -= (lU[0] * U[0] + lU[1] * U[1] + lU[2] * U[2]) * inv_rho;
    // moments: d rho = sum f, j = sum f c, S2 = sum f c c
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int cx = cq(i, 0), cy = cq(i, 1), cz = cq(i, 2);
      lf[i] = lrho + R(cx) * lj[0] + R(cy) * lj[1] + R(cz) * lj[2] + R(cx * cx) * ls2[0] + R(cy * cy) * ls2[1]
            + R(cz * cz) * ls2[2] + R(cx * cy) * ls2[3] + R(cx * cz) * ls2[4] + R(cy * cz) * ls2[5];
    }
  }
  // ---- magnetic moments: b_c = sum_i g_ic (+ S/2), Lambda_ac = g_{+a,c} - g_{-a,c}
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) lg[i * 3 + c] += lb[c];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lg[(4 + a) * 3 + c] += llam[a][c];
      lg[(1 + a) * 3 + c] -= llam[a][c];
    }
}

template <typename R, bool MOMENT>
FLAME_HD void collide_vjp(const R (&f)[kQ], const R (&g)[kM], const R (&F)[3], const R (&S)[3],
                          const R (&Jst)[3], const PhysConst<R>& k, const R (&mf)[kQ], const R (&mg)[kM],
                          R (&lf)[kQ], R (&lg)[kM], R (&lJ)[3]) {
  vjp_reverse<R, MOMENT>(vjp_forward<R, MOMENT>(f, g, F, S, Jst, k), F, k, mf, mg, lf, lg, lJ);
}

// ------------------------------------------------------------------ initial state of a node
// Deviations of the initial populations at a node (rho = 1): fluid f^mhd(0)(1, u, B) plus the
// first-order non-equilibrium stress P0 = -(c_s^2 / w)(G + G^T - 2/3 tr G I), G = grad u, and
// -F/2 first central moment; magnetic g^Hall(0)(u, B, curl b) - (1/w_B) W_i xi_ia d_a b_c - S/2 W_i
// (with u taken as zero in g^Hall(0) for electron MHD).
// G[a][c] = d u_c / d x_a, H[a][c] = d b_c / d x_a (ignored unless the flags say present).
struct InitFlags {
  bool fluid_noneq;   // add the fluid non-equilibrium stress (needs G)
  bool mag_noneq;     // add the magnetic non-equilibrium part (needs H)
  bool has_H;         // J = curl b from H (else J = 0)
  bool emhd = false;  // electron MHD: the magnetic equilibrium without the bulk velocity
};

FLAME_HD void init_node(const double (&u)[3], const double (&b)[3], const double (&G)[3][3],
                        const double (&H)[3][3], const double (&F)[3], const double (&S)[3],
                        const PhysConst<double>& k, InitFlags fl, double (&f)[kQ], double (&g)[kM]) {
  const double B[3] = {k.b0[0] + b[0], k.b0[1] + b[1], k.b0[2] + b[2]};
  double P[3][3] = {};
  if (fl.fluid_noneq) {
    const double div = G[0][0] + G[1][1] + G[2][2];
    const double s = -(1.0 / 3.0) / k.omega;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) P[p][q] = s * (G[p][q] + G[q][p] - (p == q ? 2.0 / 3.0 * div : 0.0));
  }
  const Axis<double> ax(u[0]), ay(u[1]), az(u[2]);
  const double sb = k.b0[0] * b[0] + k.b0[1] * b[1] + k.b0[2] * b[2] + 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  for (int i = 0; i < kQ; ++i) {
    const int x = cq(i, 0) + 1, y = cq(i, 1) + 1, z = cq(i, 2) + 1;
    const double ex = ax.e[x], ey = ay.e[y], ez = az.e[z];
    const double em1 = ex + (1.0 + ex) * (ey + (1.0 + ey) * ez);
    const double w = wq(i);
    double v = w * em1;
    const double bc = cq(i, 0) * b[0] + cq(i, 1) * b[1] + cq(i, 2) * b[2];
    const double b0c = cq(i, 0) * k.b0[0] + cq(i, 1) * k.b0[1] + cq(i, 2) * k.b0[2];
    v += w * 4.5 * (sb * (speed2q(i) - 1.0 / 3.0) - bc * (2.0 * b0c + bc));
    const double h0x = ax.h0[x], h0y = ay.h0[y], h0z = az.h0[z];
    const double h1x = ax.h1[x], h1y = ay.h1[y], h1z = az.h1[z];
    const double h2x = ax.h2[x], h2y = ay.h2[y], h2z = az.h2[z];
    v += P[0][0] * h2x * h0y * h0z + P[1][1] * h0x * h2y * h0z + P[2][2] * h0x * h0y * h2z
       + P[0][1] * h1x * h1y * h0z + P[0][2] * h1x * h0y * h1z + P[1][2] * h0x * h1y * h1z;
    v -= 0.5 * (F[0] * h1x * h0y * h0z + F[1] * h0x * h1y * h0z + F[2] * h0x * h0y * h1z);
    f[i] = v;
  }
  double J[3] = {0, 0, 0};
  if (fl.has_H) {
    J[0] = H[1][2] - H[2][1];
    J[1] = H[2][0] - H[0][2];
    J[2] = H[0][1] - H[1][0];
  }
  const double um = fl.emhd ? 0.0 : 1.0;
  const double V[3] = {um * u[0] - k.alpha * J[0], um * u[1] - k.alpha * J[1], um * u[2] - k.alpha * J[2]};
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c) {
      double xv = 0, xb = 0, xg = 0;
      for (int p = 0; p < 3; ++p) {
        xv += xim(i, p) * V[p];
        xb += xim(i, p) * B[p];
        xg += xim(i, p) * H[p][c];
      }
      double v = wm(i) * (b[c] + 4.0 * (xv * B[c] - xb * V[c]));
      if (fl.mag_noneq) v -= wm(i) * xg / k.omega_b;
      v -= 0.5 * wm(i) * S[c];
      g[i * 3 + c] = v;
    }
}

// Vector-Jacobian product of init_node: lf, lg = d loss / d(initial deviations) ->
// gu, gb, gG, gH = d loss / d(u, b, G, H) at the node.
FLAME_HD void init_node_vjp(const double (&u)[3], const double (&b)[3], const double (&G)[3][3],
                            const double (&H)[3][3], const double (&F)[3], const PhysConst<double>& k,
                            InitFlags fl, const double (&lf)[kQ], const double (&lg)[kM], double (&gu)[3],
                            double (&gb)[3], double (&gG)[3][3], double (&gH)[3][3]) {
  const double B[3] = {k.b0[0] + b[0], k.b0[1] + b[1], k.b0[2] + b[2]};
  for (int a = 0; a < 3; ++a) {
    gu[a] = gb[a] = 0.0;
    for (int c = 0; c < 3; ++c) gG[a][c] = gH[a][c] = 0.0;
  }
  double P[3][3] = {};
  const double s = -(1.0 / 3.0) / k.omega;
  if (fl.fluid_noneq) {
    const double div = G[0][0] + G[1][1] + G[2][2];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) P[p][q] = s * (G[p][q] + G[q][p] - (p == q ? 2.0 / 3.0 * div : 0.0));
  }
  const Axis<double> ax(u[0]), ay(u[1]), az(u[2]);
  const AxisD<double> dx(u[0]), dy(u[1]), dz(u[2]);
  double lP[6] = {0, 0, 0, 0, 0, 0};   // xx, yy, zz, xy, xz, yz
  const double fhx = -0.5 * F[0], fhy = -0.5 * F[1], fhz = -0.5 * F[2];
  for (int i = 0; i < kQ; ++i) {
    const int x = cq(i, 0) + 1, y = cq(i, 1) + 1, z = cq(i, 2) + 1;
    const double mu = lf[i];
    const double w = wq(i);
    const double ex = 1.0 + ax.e[x], ey = 1.0 + ay.e[y], ez = 1.0 + az.e[z];
    gu[0] += mu * w * dx.de[x] * ey * ez;
    gu[1] += mu * w * ex * dy.de[y] * ez;
    gu[2] += mu * w * ex * ey * dz.de[z];
    const double Bc = cq(i, 0) * B[0] + cq(i, 1) * B[1] + cq(i, 2) * B[2];
    const double c2 = speed2q(i) - 1.0 / 3.0;
    for (int d = 0; d < 3; ++d) gb[d] += mu * w * 4.5 * (B[d] * c2 - 2.0 * cq(i, d) * Bc);
    const double h0x = ax.h0[x], h0y = ay.h0[y], h0z = az.h0[z];
    const double h1x = ax.h1[x], h1y = ay.h1[y], h1z = az.h1[z];
    const double h2x = ax.h2[x], h2y = ay.h2[y], h2z = az.h2[z];
    const double d0x = dx.dh0[x], d0y = dy.dh0[y], d0z = dz.dh0[z];
    const double d1x = dx.dh1[x], d1y = dy.dh1[y], d1z = dz.dh1[z];
    lP[0] += mu * h2x * h0y * h0z;
    lP[1] += mu * h0x * h2y * h0z;
    lP[2] += mu * h0x * h0y * h2z;
    lP[3] += mu * h1x * h1y * h0z;
    lP[4] += mu * h1x * h0y * h1z;
    lP[5] += mu * h0x * h1y * h1z;
    const double qxx = P[0][0], qyy = P[1][1], qzz = P[2][2], qxy = P[0][1], qxz = P[0][2], qyz = P[1][2];
    gu[0] += mu * (qyy * d0x * h2y * h0z + qzz * d0x * h0y * h2z + qxy * d1x * h1y * h0z + qxz * d1x * h0y * h1z
                   + qyz * d0x * h1y * h1z + fhx * d1x * h0y * h0z + fhy * d0x * h1y * h0z + fhz * d0x * h0y * h1z);
    gu[1] += mu * (qxx * h2x * d0y * h0z + qzz * h0x * d0y * h2z + qxy * h1x * d1y * h0z + qxz * h1x * d0y * h1z
                   + qyz * h0x * d1y * h1z + fhx * h1x * d0y * h0z + fhy * h0x * d1y * h0z + fhz * h0x * d0y * h1z);
    gu[2] += mu * (qxx * h2x * h0y * d0z + qyy * h0x * h2y * d0z + qxy * h1x * h1y * d0z + qxz * h1x * h0y * d1z
                   + qyz * h0x * h1y * d1z + fhx * h1x * h0y * d0z + fhy * h0x * h1y * d0z + fhz * h0x * h0y * d1z);
  }
  if (fl.fluid_noneq) {
    const double ltr = lP[0] + lP[1] + lP[2];
    for (int a = 0; a < 3; ++a) gG[a][a] += s * (2.0 * lP[a] - 2.0 / 3.0 * ltr);
    gG[0][1] += s * lP[3]; gG[1][0] += s * lP[3];
    gG[0][2] += s * lP[4]; gG[2][0] += s * lP[4];
    gG[1][2] += s * lP[5]; gG[2][1] += s * lP[5];
  }
  double J[3] = {0, 0, 0};
  if (fl.has_H) {
    J[0] = H[1][2] - H[2][1];
    J[1] = H[2][0] - H[0][2];
    J[2] = H[0][1] - H[1][0];
  }
  const double V[3] = {u[0] - k.alpha * J[0], u[1] - k.alpha * J[1], u[2] - k.alpha * J[2]};
  double lV[3] = {0, 0, 0};
  for (int i = 0; i < 7; ++i)
    for (int c = 0; c < 3; ++c) {
      const double mu = lg[i * 3 + c];
      const double W = wm(i);
      double xv = 0, xb = 0;
      for (int p = 0; p < 3; ++p) {
        xv += xim(i, p) * V[p];
        xb += xim(i, p) * B[p];
      }
      gb[c] += mu * W * (1.0 + 4.0 * xv);
      lV[c] -= mu * 4.0 * W * xb;
      for (int d = 0; d < 3; ++d) {
        gb[d] -= mu * 4.0 * W * xim(i, d) * V[c];
        lV[d] += mu * 4.0 * W * xim(i, d) * B[c];
        if (fl.mag_noneq) gH[d][c] -= mu * W * xim(i, d) / k.omega_b;
      }
    }
  for (int a = 0; a < 3; ++a) gu[a] += lV[a];
  if (fl.has_H) {
    const double lJ[3] = {-k.alpha * lV[0], -k.alpha * lV[1], -k.alpha * lV[2]};
    gH[1][2] += lJ[0]; gH[2][1] -= lJ[0];
    gH[2][0] += lJ[1]; gH[0][2] -= lJ[1];
    gH[0][1] += lJ[2]; gH[1][0] -= lJ[2];
  }
}

// Periodic neighbour of a node.
FLAME_HD int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

}  // namespace flame
