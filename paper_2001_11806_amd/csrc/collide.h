// Per-cell collision operators on shifted populations.
//
// Input/output f[q] holds the shifted population f_q - w_q rho_0 in the
// compute type R.  All operators work on these small deviations directly:
// density deviation drho = sum f, momentum j = sum c f (the shift has zero
// momentum), so no large cancelling sums are ever formed in FP32.
//
// Guo forcing (cited by the paper, Sec. I): velocity u = (j + F/2)/rho_0,
// source S_q = w_q [3 (c_q - u).F + 9 (c_q.u)(c_q.F)] (c_s^2 = 1/3) with the
// (1 - omega/2) prefactor of each relaxation group.
#pragma once

#include "lattice.h"

namespace lbm {

// Internal method codes: the ABI's four, plus SRT and MRT with the
// Smagorinsky model (local shear rate).
enum { M_SRT = 0, M_TRT = 1, M_MRT = 2, M_CUMULANT = 3, M_SRT_SMAG = 4, M_MRT_SMAG = 5, M_CUMULANT_GEN = 6, M_KBC = 7,
       M_MRT_UNIT = 8 };

template <class R>
struct CollideParams {
  R rho0;
  R om;       // SRT omega / TRT even / MRT, cumulant shear
  R om_b;     // bulk
  R om_o;     // TRT odd
  R hi[4];    // orders 3..6
  R smag18;   // 18 C_S^2
  int compressible;
  const R* wall;          // wall velocity table [128][3]
  const uint32_t* links;  // per cell: bit q set when x - c_q is solid (cells next to a wall)
  int moving;             // the mask holds moving-wall types (values >= 2)
};


// Smagorinsky model (Sec. III-C "Turbulence models", Eqs. 11-14): eddy
// viscosity (C_S Delta)^2 |S| with Delta = 1 and the strain rate from the
// non-equilibrium stress, S = -3 omega / (2 rho) Pi^neq (Eq. 12).  Inserting
// |S| into omega = 2 / (6 C_S^2 |S| + 6 nu_0 + 1) (Eq. 14) gives a quadratic
// in omega whose positive root is
//   omega = 2 / (tau0 + sqrt(tau0^2 + 18 C_S^2 P / rho)),
// P = sqrt(2 Pi^neq : Pi^neq), tau0 = 1 / omega_0.  Arguments: the six
// independent components of Pi^neq.
template <class R>
__device__ __forceinline__ R smagorinsky_omega(R xx, R yy, R zz, R xy, R xz, R yz, R rho,
                                               const CollideParams<R>& p) {
  const R PP = xx * xx + yy * yy + zz * zz + R(2) * (xy * xy + xz * xz + yz * yz);
  const R P = sqrt(R(2) * PP);
  const R tau0 = R(1) / p.om;
  return R(2) / (tau0 + sqrt(tau0 * tau0 + p.smag18 * P / rho));
}

// c_q . (x, y, z) with the constant components folded away.
template <class L, class R>
__device__ __forceinline__ R cdot(int q, R x, R y, R z) {
  R s = R(0);
  if (L::c(q, 0) == 1) s += x;
  if (L::c(q, 0) == -1) s -= x;
  if (L::c(q, 1) == 1) s += y;
  if (L::c(q, 1) == -1) s -= y;
  if (L::c(q, 2) == 1) s += z;
  if (L::c(q, 2) == -1) s -= z;
  return s;
}

// Velocity bounce-back term (Sec. III-C "Boundary Conditions"): the missing
// population of link q is the cell's own outgoing opposite population plus
// 2 w_q rho_0 (c_q . u_w) / c_s^2, u_w the velocity of wall type k (row k of
// the table; row 1, the resting wall, is zero).
template <class L, class R>
__device__ __forceinline__ R wall_term(int q, int k, const R* wall, R rho0) {
  const R* u = wall + 3 * k;
  return R(6.0 * weight<L>(q)) * rho0 * cdot<L>(q, u[0], u[1], u[2]);
}

template <class L, class R>
__device__ __forceinline__ void density_momentum(const R* f, R& drho, R& jx, R& jy, R& jz) {
  drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    drho += f[q];
    if (L::c(q, 0) == 1) jx += f[q];
    if (L::c(q, 0) == -1) jx -= f[q];
    if (L::c(q, 1) == 1) jy += f[q];
    if (L::c(q, 1) == -1) jy -= f[q];
    if (L::c(q, 2) == 1) jz += f[q];
    if (L::c(q, 2) == -1) jz -= f[q];
  }
}

// ---------------------------------------------------------------- SRT
// Eq. (1): f* = f - omega (f - f^eq) + (1 - omega/2) S, f^eq from Eq. (3).
template <class L, class R, bool SMAG = false>
__device__ __forceinline__ void collide_srt(R* f, const R* F, const CollideParams<R>& p) {
  R drho, jx, jy, jz;
  density_momentum<L>(f, drho, jx, jy, jz);
  const R rho = p.rho0 + drho;
  const R rr = p.compressible ? rho : p.rho0;
  const R inv = R(1) / rr;
  const R ux = (jx + R(0.5) * F[0]) * inv, uy = (jy + R(0.5) * F[1]) * inv,
          uz = (jz + R(0.5) * F[2]) * inv;
  const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R uF3 = R(3) * (ux * F[0] + uy * F[1] + uz * F[2]);
  R om = p.om;
  if constexpr (SMAG) {
    R xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const R cu = cdot<L>(q, ux, uy, uz);
      const R d = f[q] - R(weight<L>(q)) * (drho + rr * (R(3) * cu + R(4.5) * cu * cu - usq));
      const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
      if (cx != 0) xx += d;
      if (cy != 0) yy += d;
      if (cz != 0) zz += d;
      if (cx * cy == 1) xy += d;
      if (cx * cy == -1) xy -= d;
      if (cx * cz == 1) xz += d;
      if (cx * cz == -1) xz -= d;
      if (cy * cz == 1) yz += d;
      if (cy * cz == -1) yz -= d;
    }
    om = smagorinsky_omega(xx, yy, zz, xy, xz, yz, rho, p);
  }
  const R fs = R(1) - R(0.5) * om;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const R w = R(weight<L>(q));
    const R cu = cdot<L>(q, ux, uy, uz);
    const R cF = cdot<L>(q, F[0], F[1], F[2]);
    const R feq = w * (drho + rr * (R(3) * cu + R(4.5) * cu * cu - usq));
    const R S = w * (R(3) * cF - uF3 + R(9) * cu * cF);
    f[q] = f[q] - om * (f[q] - feq) + fs * S;
  }
}

// ---------------------------------------------------------------- TRT
// Even moments relax with omega_e, odd with omega_o (Sec. III-C); written on
// the symmetric / antisymmetric parts of each (q, opp(q)) pair, where even
// moments vanish on the antisymmetric and odd moments on the symmetric part.
template <class L, class R>
__device__ __forceinline__ void collide_trt(R* f, const R* F, const CollideParams<R>& p) {
  R drho, jx, jy, jz;
  density_momentum<L>(f, drho, jx, jy, jz);
  const R rho = p.rho0 + drho;
  const R rr = p.compressible ? rho : p.rho0;
  const R inv = R(1) / rr;
  const R ux = (jx + R(0.5) * F[0]) * inv, uy = (jy + R(0.5) * F[1]) * inv,
          uz = (jz + R(0.5) * F[2]) * inv;
  const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R uF3 = R(3) * (ux * F[0] + uy * F[1] + uz * F[2]);
  const R we = p.om, wo = p.om_o;
  const R fe = R(1) - R(0.5) * we, fo = R(1) - R(0.5) * wo;
  {
    const R w = R(weight<L>(0));
    const R feq = w * (drho - rr * usq);
    f[0] = f[0] - we * (f[0] - feq) - fe * w * uF3;
  }
#pragma unroll
  for (int q = 1; q <= L::H; ++q) {
    const int o = q + L::H;
    const R w = R(weight<L>(q));
    const R cu = cdot<L>(q, ux, uy, uz);
    const R cF = cdot<L>(q, F[0], F[1], F[2]);
    const R fp = R(0.5) * (f[q] + f[o]), fm = R(0.5) * (f[q] - f[o]);
    const R ep = w * (drho + rr * (R(4.5) * cu * cu - usq));
    const R em = w * rr * R(3) * cu;
    const R sp = w * (R(9) * cu * cF - uF3);
    const R sm = w * R(3) * cF;
    const R dp = -we * (fp - ep) + fe * sp;
    const R dm = -wo * (fm - em) + fo * sm;
    f[q] += dp + dm;
    f[o] += dp - dm;
  }
}

// ---------------------------------------------------------------- MRT
// Eq. (4) in the lattice-weighted orthogonal basis built by the paper's
// Gram-Schmidt procedure.  On the tensor-product stencils D2Q9 / D3Q27 that
// basis spans, group by group, the same subspaces as the products
// p_a(c_x) p_b(c_y) p_c(c_z) of the 1-D weighted-orthogonal polynomials
// p_0 = 1, p_1 = c, p_2 = 3c^2 - 1 (norms 1, 1/3, 2), and the relaxation
// depends only on those subspaces.  So the moment transform factorises into
// three 1-D 3-point transforms per axis, forward and back:
//   A_k = sum_q H_k(c_q) f_q,    f*_q = f_q + w_q sum_k H_k(c_q) gamma_k,
//   gamma_k = -omega_g (A_k - A_k^eq) / |H_k|^2 + (1 - omega_g/2) sigma_k,
// where sigma_k are the coefficients of the Guo source in the same basis.
// Groups: order 0, 1 conserved; order 2 split into shear (off-diagonal and
// traceless diagonal, omega) and bulk (trace, omega_b); order n >= 3 hi[n-3].
// Eq. (3) has no component of order >= 3 on these stencils.
// Hermite coefficients a[i][j][k] = sum_q h_i(c_x) h_j(c_y) h_k(c_z) f_q of the
// shifted populations, h_0 = 1, h_1 = c, h_2 = 3c^2 - 1 (k = 0 only in 2-D):
// per axis (v-, v0, v+) -> (sum, v+ - v-, 2v- - v0 + 2v+).
template <class L, class R>
__device__ __forceinline__ void mrt_forward(const R* f, R (&a)[3][3][(L::DIM == 3) ? 3 : 1]) {
  constexpr int D = L::DIM;
  constexpr int NK = (D == 3) ? 3 : 1;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) a[i][j][k] = f[qindex<L>(i - 1, j - 1, D == 3 ? k - 1 : 0)];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const R m = a[0][j][k], z = a[1][j][k], pp = a[2][j][k];
      a[0][j][k] = m + z + pp;
      a[1][j][k] = pp - m;
      a[2][j][k] = R(2) * (m + pp) - z;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const R m = a[i][0][k], z = a[i][1][k], pp = a[i][2][k];
      a[i][0][k] = m + z + pp;
      a[i][1][k] = pp - m;
      a[i][2][k] = R(2) * (m + pp) - z;
    }
  if constexpr (D == 3) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R m = a[i][j][0], z = a[i][j][NK > 1 ? 1 : 0], pp = a[i][j][NK - 1];
        a[i][j][0] = m + z + pp;
        a[i][j][NK > 1 ? 1 : 0] = pp - m;
        a[i][j][NK - 1] = R(2) * (m + pp) - z;
      }
  }
}

// gamma_k of orders 0..2 written over those coefficients of a (the others
// are left alone): conserved orders 0, 1 (rate 0, Guo sigma = 3 F_a), the
// shear group (off-diagonal and traceless diagonal, omega) and the bulk
// trace (omega_b); rr = rho (compressible) or rho_0.
template <class L, class R>
__device__ __forceinline__ void mrt_gamma2(R (&a)[3][3][(L::DIM == 3) ? 3 : 1], const R* F, R rr, R ux, R uy,
                                           R uz, R om, R omb) {
  constexpr int D = L::DIM;
  constexpr int NK = (D == 3) ? 3 : 1;
  const R fs = R(1) - R(0.5) * om, fb = R(1) - R(0.5) * omb;
  // order 0 and 1: conserved (rate 0); the source gives sigma = 3 F_a
  a[0][0][0] = R(0);
  a[1][0][0] = R(3) * F[0];
  a[0][1][0] = R(3) * F[1];
  if constexpr (D == 3) a[0][0][1] = R(3) * F[2];
  // order 2, off-diagonal: |H|^2 = 1/9, A^eq = rr u_a u_b, sigma = 9 (u_a F_b + u_b F_a)
  {
    a[1][1][0] = -om * R(9) * (a[1][1][0] - rr * ux * uy) + fs * R(9) * (ux * F[1] + uy * F[0]);
    if constexpr (D == 3) {
      a[1][0][1] = -om * R(9) * (a[1][0][1] - rr * ux * uz) + fs * R(9) * (ux * F[2] + uz * F[0]);
      a[0][1][1] = -om * R(9) * (a[0][1][1] - rr * uy * uz) + fs * R(9) * (uy * F[2] + uz * F[1]);
    }
  }
  // order 2, diagonal: |H|^2 = 2, A^eq = 3 rr u_a^2, sigma = 3 u_a F_a;
  // trace part relaxes with omega_b, traceless part with omega
  {
    R An[3], sg[3];
    An[0] = a[2][0][0] - R(3) * rr * ux * ux;
    An[1] = a[0][2][0] - R(3) * rr * uy * uy;
    An[2] = (D == 3) ? a[0][0][NK - 1] - R(3) * rr * uz * uz : R(0);
    sg[0] = R(3) * ux * F[0];
    sg[1] = R(3) * uy * F[1];
    sg[2] = R(3) * uz * F[2];
    const R invD = R(1) / R(D);
    const R mA = (An[0] + An[1] + An[2]) * invD;
    const R mS = (sg[0] + sg[1] + sg[2]) * invD;
    R g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      g[c] = -R(0.5) * (om * (An[c] - mA) + omb * mA) + fs * (sg[c] - mS) + fb * mS;
    a[2][0][0] = g[0];
    a[0][2][0] = g[1];
    if constexpr (D == 3) a[0][0][NK - 1] = g[2];
  }
}

template <class L, class R, bool SMAG = false>
__device__ __forceinline__ void collide_mrt(R* f, const R* F, const CollideParams<R>& p) {
  constexpr int D = L::DIM;
  constexpr int NK = (D == 3) ? 3 : 1;
  R a[3][3][NK];
  mrt_forward<L>(f, a);
  // a[i][j][k] now holds A for Hermite orders (i, j, k) (k = 0 in 2-D)
  const R drho = a[0][0][0];
  const R rho = p.rho0 + drho;
  const R rr = p.compressible ? rho : p.rho0;
  const R inv = R(1) / rr;
  const R ux = (a[1][0][0] + R(0.5) * F[0]) * inv;
  const R uy = (a[0][1][0] + R(0.5) * F[1]) * inv;
  const R uz = (D == 3) ? (a[0][0][NK > 1 ? 1 : 0] + R(0.5) * F[2]) * inv : R(0);
  R om = p.om;
  if constexpr (SMAG) {
    // Pi^neq from the Hermite coefficients: off-diagonal A_ab - rr u_a u_b,
    // diagonal (A_aa - 3 rr u_a^2) / 3 (the neq mass is zero)
    const R xy = a[1][1][0] - rr * ux * uy;
    const R xx = (a[2][0][0] - R(3) * rr * ux * ux) * R(1.0 / 3.0);
    const R yy = (a[0][2][0] - R(3) * rr * uy * uy) * R(1.0 / 3.0);
    R zz = R(0), xz = R(0), yz = R(0);
    if constexpr (D == 3) {
      zz = (a[0][0][NK - 1] - R(3) * rr * uz * uz) * R(1.0 / 3.0);
      xz = a[1][0][1] - rr * ux * uz;
      yz = a[0][1][1] - rr * uy * uz;
    }
    om = smagorinsky_omega(xx, yy, zz, xy, xz, yz, rho, p);
  }
  // gamma in place
  mrt_gamma2<L>(a, F, rr, ux, uy, uz, om, p.om_b);
  // orders >= 3: A^eq = 0, no source
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int kk = (D == 3) ? k : 0;
        const int n = i + j + kk;
        if (n >= 3) {
          const R invn = R((i == 1 ? 3.0 : (i == 2 ? 0.5 : 1.0)) * (j == 1 ? 3.0 : (j == 2 ? 0.5 : 1.0)) *
                           (kk == 1 ? 3.0 : (kk == 2 ? 0.5 : 1.0)));
          a[i][j][k] = -p.hi[n - 3] * invn * a[i][j][k];
        }
      }
  // back transforms with the 1-D weights (1/6, 2/3, 1/6):
  // (g0, g1, g2) -> w(-1)(g0 - g1 + 2g2), w(0)(g0 - g2), w(+1)(g0 + g1 + 2g2)
  if constexpr (D == 3) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R g0 = a[i][j][0], g1 = a[i][j][NK > 1 ? 1 : 0], g2 = a[i][j][NK - 1];
        a[i][j][0] = R(1.0 / 6.0) * (g0 - g1 + R(2) * g2);
        a[i][j][NK > 1 ? 1 : 0] = R(2.0 / 3.0) * (g0 - g2);
        a[i][j][NK - 1] = R(1.0 / 6.0) * (g0 + g1 + R(2) * g2);
      }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const R g0 = a[i][0][k], g1 = a[i][1][k], g2 = a[i][2][k];
      a[i][0][k] = R(1.0 / 6.0) * (g0 - g1 + R(2) * g2);
      a[i][1][k] = R(2.0 / 3.0) * (g0 - g2);
      a[i][2][k] = R(1.0 / 6.0) * (g0 + g1 + R(2) * g2);
    }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const R g0 = a[0][j][k], g1 = a[1][j][k], g2 = a[2][j][k];
      a[0][j][k] = R(1.0 / 6.0) * (g0 - g1 + R(2) * g2);
      a[1][j][k] = R(2.0 / 3.0) * (g0 - g2);
      a[2][j][k] = R(1.0 / 6.0) * (g0 + g1 + R(2) * g2);
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int q = qindex<L>(i - 1, j - 1, D == 3 ? k - 1 : 0);
        f[q] += a[i][j][k];
      }
}

// 1-D back transforms of a line with the 1-D weights (1/6, 2/3, 1/6):
// (g0, g1, g2) -> (w-(g0 - g1 + 2g2), w0(g0 - g2), w+(g0 + g1 + 2g2)), and the
// same for lines whose last one or two entries are zero (skipped, not added:
// the compiler may not drop an addition of zero under IEEE rules).
template <class R>
__device__ __forceinline__ void back_line3(R g0, R g1, R g2, R* o) {
  o[0] = R(1.0 / 6.0) * (g0 - g1 + R(2) * g2);
  o[1] = R(2.0 / 3.0) * (g0 - g2);
  o[2] = R(1.0 / 6.0) * (g0 + g1 + R(2) * g2);
}
template <class R>
__device__ __forceinline__ void back_line2(R g0, R g1, R* o) {
  o[0] = R(1.0 / 6.0) * (g0 - g1);
  o[1] = R(2.0 / 3.0) * g0;
  o[2] = R(1.0 / 6.0) * (g0 + g1);
}
template <class R>
__device__ __forceinline__ void back_line1(R g0, R* o) {
  o[0] = R(1.0 / 6.0) * g0;
  o[1] = R(2.0 / 3.0) * g0;
  o[2] = o[0];
}

// MRT with every rate of order >= 3 equal to 1 (the Kolmogorov workload):
// Eq. (4) in the basis of collide_mrt, where relaxing those orders at rate 1
// leaves them zero after the collision (Eq. (3) has no component there).  So
// f* is rebuilt from its coefficients of orders <= 2 alone,
//   f*_q = w_q sum_{|k| <= 2} H_k(c_q) c_k,  c_k = A_k / |H_k|^2 + gamma_k,
// which needs 10 of the 27 forward coefficients (the compiler drops the
// rest) and a back transform over lines that are mostly zero: the same
// operator as collide_mrt with hi = 1 in about two thirds of its arithmetic.
template <class L, class R>
__device__ __forceinline__ void collide_mrt_unit(R* f, const R* F, const CollideParams<R>& p) {
  constexpr int D = L::DIM;
  constexpr int NK = (D == 3) ? 3 : 1;
  R a[3][3][NK];
  mrt_forward<L>(f, a);
  const R drho = a[0][0][0];
  const R rho = p.rho0 + drho;
  const R rr = p.compressible ? rho : p.rho0;
  const R inv = R(1) / rr;
  const R ux = (a[1][0][0] + R(0.5) * F[0]) * inv;
  const R uy = (a[0][1][0] + R(0.5) * F[1]) * inv;
  const R uz = (D == 3) ? (a[0][0][NK > 1 ? 1 : 0] + R(0.5) * F[2]) * inv : R(0);
  // A_k / |H_k|^2 of orders 1 and 2 before gamma overwrites them
  const R s100 = R(3) * a[1][0][0], s010 = R(3) * a[0][1][0];
  const R s110 = R(9) * a[1][1][0], s200 = R(0.5) * a[2][0][0], s020 = R(0.5) * a[0][2][0];
  R s001 = R(0), s101 = R(0), s011 = R(0), s002 = R(0);
  if constexpr (D == 3) {
    s001 = R(3) * a[0][0][1];
    s101 = R(9) * a[1][0][1];
    s011 = R(9) * a[0][1][1];
    s002 = R(0.5) * a[0][0][2];
  }
  mrt_gamma2<L>(a, F, rr, ux, uy, uz, p.om, p.om_b);
  const R c000 = drho;   // gamma = 0: the mass is conserved
  const R c100 = s100 + a[1][0][0], c010 = s010 + a[0][1][0];
  const R c110 = s110 + a[1][1][0], c200 = s200 + a[2][0][0], c020 = s020 + a[0][2][0];
  if constexpr (D == 3) {
    const R c001 = s001 + a[0][0][1], c101 = s101 + a[1][0][1], c011 = s011 + a[0][1][1];
    const R c002 = s002 + a[0][0][2];
    // pass z: E[i][j][kk] for the (i, j) lines with a nonzero entry
    R e00[3], e10[3], e01[3], e11[3], e20[3], e02[3];
    back_line3(c000, c001, c002, e00);
    back_line2(c100, c101, e10);
    back_line2(c010, c011, e01);
    back_line1(c110, e11);
    back_line1(c200, e20);
    back_line1(c020, e02);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      // pass y: G[i][jj] for this kk
      R g0[3], g1[3], g2[3];
      back_line3(e00[kk], e01[kk], e02[kk], g0);
      back_line2(e10[kk], e11[kk], g1);
      back_line1(e20[kk], g2);
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        R o[3];   // pass x
        back_line3(g0[jj], g1[jj], g2[jj], o);
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) f[qindex<L>(ii - 1, jj - 1, kk - 1)] = o[ii];
      }
    }
  } else {
    R g0[3], g1[3], g2[3];   // pass y
    back_line3(c000, c010, c020, g0);
    back_line2(c100, c110, g1);
    back_line1(c200, g2);
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      R o[3];   // pass x
      back_line3(g0[jj], g1[jj], g2[jj], o);
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) f[qindex<L>(ii - 1, jj - 1, 0)] = o[ii];
    }
  }
}

// ---------------------------------------------------------------- MRT (general stencil)
// Eq. (4) with the weighted-orthogonal basis built exactly as Sec. III-A/C
// describe it: independent monomials x^a y^b z^c (a, b, c <= 2, rows that
// vanish on the stencil dropped), second order split into shear (x^2 - y^2,
// x^2 - z^2, off-diagonal) and bulk (x^2 + y^2 + z^2), ordered by order, then
// Gram-Schmidt with <p, r>_w = sum_q w_q p(c_q) r(c_q).  The basis is computed
// at compile time (constexpr), so every matrix entry is an immediate and the
// zero entries cost nothing.  Used for D3Q19, whose basis is not a tensor
// product.
template <int Q>
struct MrtBasis {
  double m[Q][Q];      // row k: polynomial k evaluated on the directions
  double inv_norm[Q];  // 1 / sum_q w_q m[k][q]^2
  int group[Q];        // 0 conserved, 1 shear, 2 bulk, n >= 3: order n
};

__host__ __device__ constexpr double ipow(int v, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= v;
  return r;
}

template <class L>
__host__ __device__ constexpr double mono(int q, int a, int b, int c) {
  return ipow(L::c(q, 0), a) * ipow(L::c(q, 1), b) * ipow(L::c(q, 2), c);
}

template <class L>
__host__ __device__ constexpr MrtBasis<L::Q> make_mrt_basis() {
  MrtBasis<L::Q> B{};
  double raw[L::Q][L::Q] = {};
  int n = 0;
  auto add_mono = [&](int a, int b, int c, int grp) {
    bool any = false;
    for (int q = 0; q < L::Q; ++q) any = any || mono<L>(q, a, b, c) != 0.0;
    if (!any || n >= L::Q) return;
    for (int q = 0; q < L::Q; ++q) raw[n][q] = mono<L>(q, a, b, c);
    B.group[n++] = grp;
  };
  add_mono(0, 0, 0, 0);
  add_mono(1, 0, 0, 0);
  add_mono(0, 1, 0, 0);
  if (L::DIM == 3) add_mono(0, 0, 1, 0);
  // second order: shear differences and off-diagonals, then bulk
  for (int k = 1; k < L::DIM; ++k) {
    for (int q = 0; q < L::Q; ++q) raw[n][q] = mono<L>(q, 2, 0, 0) - (k == 1 ? mono<L>(q, 0, 2, 0) : mono<L>(q, 0, 0, 2));
    B.group[n++] = 1;
  }
  add_mono(1, 1, 0, 1);
  if (L::DIM == 3) {
    add_mono(1, 0, 1, 1);
    add_mono(0, 1, 1, 1);
  }
  for (int q = 0; q < L::Q; ++q)
    raw[n][q] = mono<L>(q, 2, 0, 0) + mono<L>(q, 0, 2, 0) + (L::DIM == 3 ? mono<L>(q, 0, 0, 2) : 0.0);
  B.group[n++] = 2;
  for (int order = 3; order <= 2 * L::DIM; ++order)
    for (int a = 0; a <= 2; ++a)
      for (int b = 0; b <= 2; ++b)
        for (int c = 0; c <= (L::DIM == 3 ? 2 : 0); ++c)
          if (a + b + c == order) add_mono(a, b, c, order);
  // weighted Gram-Schmidt
  for (int k = 0; k < L::Q; ++k) {
    for (int j = 0; j < k; ++j) {
      double num = 0.0, den = 0.0;
      for (int q = 0; q < L::Q; ++q) {
        num += weight<L>(q) * raw[k][q] * raw[j][q];
        den += weight<L>(q) * raw[j][q] * raw[j][q];
      }
      for (int q = 0; q < L::Q; ++q) raw[k][q] -= num / den * raw[j][q];
    }
  }
  for (int k = 0; k < L::Q; ++k) {
    double nrm = 0.0;
    for (int q = 0; q < L::Q; ++q) {
      // snap roundoff of exactly-zero entries so they fold away
      const double v = raw[k][q];
      B.m[k][q] = (v < 1e-13 && v > -1e-13) ? 0.0 : v;
      nrm += weight<L>(q) * B.m[k][q] * B.m[k][q];
    }
    B.inv_norm[k] = 1.0 / nrm;
  }
  return B;
}

template <class L, class R, bool SMAG = false>
__device__ __forceinline__ void collide_mrt_gs(R* f, const R* F, const CollideParams<R>& p) {
  constexpr MrtBasis<L::Q> B = make_mrt_basis<L>();
  R drho, jx, jy, jz;
  density_momentum<L>(f, drho, jx, jy, jz);
  const R rho = p.rho0 + drho;
  const R rr = p.compressible ? rho : p.rho0;
  const R inv = R(1) / rr;
  const R ux = (jx + R(0.5) * F[0]) * inv, uy = (jy + R(0.5) * F[1]) * inv,
          uz = (jz + R(0.5) * F[2]) * inv;
  const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R uF3 = R(3) * (ux * F[0] + uy * F[1] + uz * F[2]);
  R neq[L::Q], src[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const R w = R(weight<L>(q));
    const R cu = cdot<L>(q, ux, uy, uz);
    const R cF = cdot<L>(q, F[0], F[1], F[2]);
    neq[q] = f[q] - w * (drho + rr * (R(3) * cu + R(4.5) * cu * cu - usq));
    src[q] = w * (R(3) * cF - uF3 + R(9) * cu * cF);
  }
  R om = p.om;
  if constexpr (SMAG) {
    R xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
      if (cx != 0) xx += neq[q];
      if (cy != 0) yy += neq[q];
      if (cz != 0) zz += neq[q];
      if (cx * cy == 1) xy += neq[q];
      if (cx * cy == -1) xy -= neq[q];
      if (cx * cz == 1) xz += neq[q];
      if (cx * cz == -1) xz -= neq[q];
      if (cy * cz == 1) yz += neq[q];
      if (cy * cz == -1) yz -= neq[q];
    }
    om = smagorinsky_omega(xx, yy, zz, xy, xz, yz, rho, p);
  }
  R gam[L::Q];
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const int grp = B.group[k];
    R a = R(0), b = R(0);
    if (grp != 0) {
#pragma unroll
      for (int q = 0; q < L::Q; ++q)
        if (B.m[k][q] != 0.0) a += R(B.m[k][q]) * neq[q];
    }
    // the Guo source has no component of order >= 3
    if (k > 0 && grp <= 2) {
#pragma unroll
      for (int q = 0; q < L::Q; ++q)
        if (B.m[k][q] != 0.0) b += R(B.m[k][q]) * src[q];
    }
    const R rate = grp == 0 ? R(0) : (grp == 1 ? om : (grp == 2 ? p.om_b : p.hi[grp - 3]));
    gam[k] = (-rate * a + (R(1) - R(0.5) * rate) * b) * R(B.inv_norm[k]);
  }
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    R d = R(0);
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
      if (B.m[k][q] != 0.0) d += R(B.m[k][q]) * gam[k];
    f[q] += R(weight<L>(q)) * d;
  }
}

// ---------------------------------------------------------------- cumulant
// Cumulant collision (Eq. 9, Sec. III-B) for the case where every rate of
// order >= 3 is 1.  Then all post-collision cumulants of order >= 3 vanish:
// the post-collision state is the discrete distribution whose cumulant
// generating function is quadratic, ln rho + u.xi + xi^T K* xi / 2, i.e. its
// central moments are Gaussian (Isserlis): c_200 = K_xx,
// c_220 = K_xx K_yy + 2 K_xy^2, c_211 = K_xx K_yz + 2 K_xy K_xz, c_222 = ...,
// all odd ones zero.  Moments with exponents <= 2 per axis map back to
// populations by a per-axis 3-point transform about the mean u_a.
// Second-order cumulants: K = Pi/rho - u u^T; shear part (off-diagonal and
// traceless diagonal) relaxes with omega, the trace with omega_b, towards the
// Maxwellian value c_s^2 I.
//
// Arithmetic layout (all in the compute type, on small quantities only):
//   - the ten raw moments of order <= 2 come from per-axis 3-point sums of
//     the shifted populations (x, then y, then z), sharing partial sums;
//   - K* = c_s^2 I + Dv; the central moments are C* = C_w + dC with C_w the
//     lattice-weight moments (a product of (1, 0, c_s^2) per axis) and dC
//     the small deviations;
//   - the back-transform is done in deviation form, one axis at a time:
//     E_1 = T_z(u_z)[dC] + (T_z(u_z) - T_z(0))[C_w], then the same along y
//     and x, where (T(v) - T(0)) of (1, 0, c_s^2) is the 1-D equilibrium
//     deviation dphi(v) = ((v^2 - v)/2, -v^2, (v^2 + v)/2); the result
//     E_3 = T_u[C*] - w, so f*_q - w_q rho_0 = rho E_3 + drho w_q (the last
//     pass carries the factor rho and the drho w_q term);
//   - zero entries of dC are skipped explicitly (the compiler may not fold
//     x * 0 under IEEE rules).

// Per-axis coefficients of the central-moment -> population transform with
// mean v, scaled by s: for the central moments (k0, k1, k2) about v,
//   f(-1) = s [(v^2 - v)/2 k0 + (v - 1/2) k1 + k2/2]
//   f( 0) = s [(1 - v^2) k0 - 2 v k1 - k2]
//   f(+1) = s [(v^2 + v)/2 k0 + (v + 1/2) k1 + k2/2]
template <class R>
struct CmAxis {
  R am, a0, ap, bm, b0, bp, h, m;  // k0 and k1 coefficients; k2 coefficients s/2 and -s
  R dm, dz, dp;                    // s dphi(v)
};

template <class R>
__device__ __forceinline__ CmAxis<R> cm_axis(R v, R s) {
  CmAxis<R> a;
  const R v2 = v * v;
  const R hs = R(0.5) * s;
  a.dm = hs * (v2 - v);
  a.dz = -s * v2;
  a.dp = hs * (v2 + v);
  a.am = a.dm;
  a.a0 = s - s * v2;
  a.ap = a.dp;
  a.bm = s * v - hs;
  a.b0 = R(-2) * s * v;
  a.bp = s * v + hs;
  a.h = hs;
  a.m = -s;
  return a;
}

// dense line: outputs (f(-1), f(0), f(+1)) into o[0..2]
template <class R>
__device__ __forceinline__ void cm_line(const CmAxis<R>& a, R k0, R k1, R k2, R* o) {
  const R hk2 = a.h * k2;
  o[0] = a.am * k0 + (a.bm * k1 + hk2);
  o[1] = a.a0 * k0 + (a.b0 * k1 + a.m * k2);
  o[2] = a.ap * k0 + (a.bp * k1 + hk2);
}
// unscaled lines with a zero pattern (s = 1)
template <class R>
__device__ __forceinline__ void cm_line_k1(const CmAxis<R>& a, R k1, R* o) {
  o[0] = a.bm * k1;
  o[1] = a.b0 * k1;
  o[2] = a.bp * k1;
}
template <class R>
__device__ __forceinline__ void cm_line_k0k2(const CmAxis<R>& a, R k0, R k2, R* o) {
  const R hk2 = R(0.5) * k2;
  o[0] = a.am * k0 + hk2;
  o[1] = a.a0 * k0 - k2;
  o[2] = a.ap * k0 + hk2;
}
// the same plus cw dphi(v), the image of the weight moments cw (1, 0, c_s^2)
// (each term formed separately: nothing of size cw is added and removed)
template <class R>
__device__ __forceinline__ void cm_line_k0k2_w(const CmAxis<R>& a, R k0, R k2, R cw, R* o) {
  const R hk2 = R(0.5) * k2;
  o[0] = a.am * k0 + (cw * a.dm + hk2);
  o[1] = a.a0 * k0 + (cw * a.dz - k2);
  o[2] = a.ap * k0 + (cw * a.dp + hk2);
}

template <class L, class R>
__device__ __forceinline__ void collide_cumulant(R* f, const R* /*F*/, const CollideParams<R>& p) {
  constexpr int D = L::DIM;
  constexpr int NK = (D == 3) ? 3 : 1;
  // 1-D weights (1/6, 2/3, 1/6) and c_s^2 = 1/3 as constants of the compute
  // type that keep the weight identities exact as real numbers: the centre
  // weight is 2/3 rounded, the side weights are (1 - that) / 2 and c_s^2 is
  // twice a side weight (both exact in R, by Sterbenz's lemma and a power-of-
  // two scaling).  Rounding 1/6 and 2/3 separately would leave
  // sum w = 1 + 3e-8 in FP32; that factor multiplies the smooth fields rho,
  // rho u and drho in every cell and step, a coherent mass and momentum
  // source that grows the FP32 velocity error linearly in time.  With the
  // identities exact, what remains of the arithmetic error is rounding noise.
  constexpr R w1c = R(2.0 / 3.0);
  constexpr R w1s = (R(1) - w1c) * R(0.5);
  constexpr R cs2 = R(2) * w1s;
  constexpr R w1[3] = {w1s, w1c, w1s};
  // ---- raw moments of order <= 2 by per-axis sums; index i = c + 1
  R X0[3][NK], X1[3][NK], X2[3][NK];   // x pass: sum, f+ - f-, f+ + f- along x
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int z = D == 3 ? k - 1 : 0;
      const R a = f[qindex<L>(-1, j - 1, z)], b = f[qindex<L>(0, j - 1, z)], c = f[qindex<L>(1, j - 1, z)];
      X2[j][k] = c + a;
      X1[j][k] = c - a;
      X0[j][k] = X2[j][k] + b;
    }
  R Y00[NK], Y01[NK], Y02[NK], Y10[NK], Y11[NK], Y20[NK];  // y pass, moments x^a y^b
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    Y02[k] = X0[2][k] + X0[0][k];
    Y01[k] = X0[2][k] - X0[0][k];
    Y00[k] = Y02[k] + X0[1][k];
    Y11[k] = X1[2][k] - X1[0][k];
    Y10[k] = (X1[2][k] + X1[0][k]) + X1[1][k];
    Y20[k] = (X2[2][k] + X2[0][k]) + X2[1][k];
  }
  R drho, jx, jy, jz = R(0), Pxx, Pyy, Pzz = R(0), Pxy, Pxz = R(0), Pyz = R(0);
  if constexpr (D == 3) {   // z pass
    const R m002 = Y00[2] + Y00[0];
    jz = Y00[2] - Y00[0];
    drho = m002 + Y00[1];
    Pzz = m002;
    jy = (Y01[2] + Y01[0]) + Y01[1];
    Pyz = Y01[2] - Y01[0];
    jx = (Y10[2] + Y10[0]) + Y10[1];
    Pxz = Y10[2] - Y10[0];
    Pyy = (Y02[2] + Y02[0]) + Y02[1];
    Pxx = (Y20[2] + Y20[0]) + Y20[1];
    Pxy = (Y11[2] + Y11[0]) + Y11[1];
  } else {
    drho = Y00[0];
    jx = Y10[0];
    jy = Y01[0];
    Pxx = Y20[0];
    Pyy = Y02[0];
    Pxy = Y11[0];
  }
  const R rho = p.rho0 + drho;
  const R inv = R(1) / rho;
  const R u[3] = {jx * inv, jy * inv, jz * inv};
  // ---- relaxed second-order cumulant deviations from c_s^2 I
  // (shift: sum c_a c_b w rho_0 = c_s^2 rho_0 delta)
  const R Kxx = (Pxx - drho * cs2) * inv - u[0] * u[0];
  const R Kyy = (Pyy - drho * cs2) * inv - u[1] * u[1];
  const R Kzz = (D == 3) ? (Pzz - drho * cs2) * inv - u[2] * u[2] : R(0);
  const R tr = (Kxx + Kyy + Kzz) * (R(1) / R(D));
  const R ks = R(1) - p.om, kb = R(1) - p.om_b;
  const R Dxx = ks * (Kxx - tr) + kb * tr;
  const R Dyy = ks * (Kyy - tr) + kb * tr;
  const R Dxy = ks * (Pxy * inv - u[0] * u[1]);
  // ---- back-transform in deviation form
  const CmAxis<R> ay = cm_axis<R>(u[1], R(1));
  const CmAxis<R> ax = cm_axis<R>(u[0], rho);   // last pass carries rho
  // per-x-population term of the last pass: rho dphi_x + drho w1
  const R gx[3] = {ax.dm + drho * w1[0], ax.dz + drho * w1[1], ax.dp + drho * w1[2]};
  if constexpr (D == 3) {
    const R Dzz = ks * (Kzz - tr) + kb * tr;
    const R Dxz = ks * (Pxz * inv - u[0] * u[2]);
    const R Dyz = ks * (Pyz * inv - u[1] * u[2]);
    // nonzero central-moment deviations beyond order 2 (Isserlis)
    const R c220 = cs2 * (Dxx + Dyy) + Dxx * Dyy + R(2) * Dxy * Dxy;
    const R c202 = cs2 * (Dxx + Dzz) + Dxx * Dzz + R(2) * Dxz * Dxz;
    const R c022 = cs2 * (Dyy + Dzz) + Dyy * Dzz + R(2) * Dyz * Dyz;
    const R c211 = (cs2 + Dxx) * Dyz + R(2) * Dxy * Dxz;
    const R c121 = (cs2 + Dyy) * Dxz + R(2) * Dxy * Dyz;
    const R c112 = (cs2 + Dzz) * Dxy + R(2) * Dxz * Dyz;
    const R c222 = cs2 * cs2 * (Dxx + Dyy + Dzz) + cs2 * (Dxx * Dyy + Dxx * Dzz + Dyy * Dzz) + Dxx * Dyy * Dzz +
                   R(2) * (cs2 + Dxx) * Dyz * Dyz + R(2) * (cs2 + Dyy) * Dxz * Dxz +
                   R(2) * (cs2 + Dzz) * Dxy * Dxy + R(8) * Dxy * Dxz * Dyz;
    const CmAxis<R> az = cm_axis<R>(u[2], R(1));
    // pass z: E[i][j][kk], i, j exponents in x, y; kk population in z.
    // C_w lines (i, j in {0, 2}) add cw_i cw_j dphi_z.
    R E[3][3][3];
    {
      const R hz = R(0.5) * Dzz;   // line (0, 0): (0, 0, Dzz) + dphi_z
      E[0][0][0] = hz + az.dm;
      E[0][0][1] = az.dz - Dzz;
      E[0][0][2] = hz + az.dp;
    }
    cm_line_k1(az, Dyz, E[0][1]);
    cm_line_k1(az, Dxz, E[1][0]);
    cm_line_k1(az, c121, E[1][2]);
    cm_line_k1(az, c211, E[2][1]);
    cm_line_k0k2(az, Dxy, c112, E[1][1]);
    cm_line_k0k2_w(az, Dyy, c022, cs2, E[0][2]);
    cm_line_k0k2_w(az, Dxx, c202, cs2, E[2][0]);
    cm_line_k0k2_w(az, c220, c222, cs2 * cs2, E[2][2]);
    // pass y: lines (i, kk) over the y exponent; C_w rows i in {0, 2} add
    // cw_i w1_kk dphi_y
    R G[3][3][3];   // G[i][jj][kk]
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        R o[3];
        cm_line(ay, E[i][0][kk], E[i][1][kk], E[i][2][kk], o);
        if (i != 1) {
          const R cw = (i == 0 ? R(1) : cs2) * w1[kk];
          o[0] += cw * ay.dm;
          o[1] += cw * ay.dz;
          o[2] += cw * ay.dp;
        }
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) G[i][jj][kk] = o[jj];
      }
    // pass x (scaled by rho) plus (rho dphi_x + drho w1) w1_jj w1_kk
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        R o[3];
        cm_line(ax, G[0][jj][kk], G[1][jj][kk], G[2][jj][kk], o);
        const R ww = w1[jj] * w1[kk];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) f[qindex<L>(ii - 1, jj - 1, kk - 1)] = o[ii] + gx[ii] * ww;
      }
  } else {
    const R c220 = cs2 * (Dxx + Dyy) + Dxx * Dyy + R(2) * Dxy * Dxy;
    // pass y: lines over i (x exponent): (0, 0, Dyy) + dphi_y, (0, Dxy, 0), (Dxx, 0, c220) + c_s^2 dphi_y
    R G[3][3];
    {
      const R hy = R(0.5) * Dyy;
      G[0][0] = hy + ay.dm;
      G[0][1] = ay.dz - Dyy;
      G[0][2] = hy + ay.dp;
    }
    cm_line_k1(ay, Dxy, G[1]);
    cm_line_k0k2_w(ay, Dxx, c220, cs2, G[2]);
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      R o[3];
      cm_line(ax, G[0][jj], G[1][jj], G[2][jj], o);
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) f[qindex<L>(ii - 1, jj - 1, 0)] = o[ii] + gx[ii] * w1[jj];
    }
  }
}

// ---------------------------------------------------------------- cumulant, general rates
// Cumulant collision (Eq. 9, Sec. III-B) with arbitrary rates for orders 3..6.
// populations -> central moments c (per-axis 3-point transforms about u)
// -> cumulants: with the first central moments zero, kappa_S is the sum over
// set partitions of S into blocks of size >= 2 of
// (-1)^(k-1) (k-1)! prod c_B (k blocks); orders 2 and 3 equal the central
// moments.  Relaxation as in the unit-rate kernel, kappa*_n = (1 - omega_n)
// kappa_n for n >= 3; the inverse relation (all coefficients +1) rebuilds the
// central moments and the back-transform the populations.  Computed in FP64
// for every storage type: the order 4-6 relations subtract products of
// O(c_s^4) terms.
template <class L, class R>
__device__ __forceinline__ void collide_cumulant_general(R* f, const R* /*F*/, const CollideParams<R>& p) {
  constexpr int D = L::DIM;
  constexpr int NK = (D == 3) ? 3 : 1;
  constexpr double cs2 = 1.0 / 3.0;
  const double rho0 = (double)p.rho0;
  double c[3][3][NK];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int q = qindex<L>(i - 1, j - 1, D == 3 ? k - 1 : 0);
        c[i][j][k] = (double)f[q] + weight<L>(q) * rho0;
      }
  double rho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const double v = c[i][j][k];
        rho += v;
        jx += (i - 1) * v;
        jy += (j - 1) * v;
        if constexpr (D == 3) jz += (k - 1) * v;
      }
  const double inv = 1.0 / rho;
  const double u[3] = {jx * inv, jy * inv, jz * inv};
  // forward transforms: (f-, f0, f+) -> central moments about v
  auto fwd = [](double& a, double& b, double& e, double v) {
    const double m0 = a + b + e, m1 = e - a, m2 = e + a;
    a = m0;
    b = m1 - v * m0;
    e = m2 - 2.0 * v * m1 + v * v * m0;
  };
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < NK; ++k) fwd(c[0][j][k], c[1][j][k], c[2][j][k], u[0]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < NK; ++k) fwd(c[i][0][k], c[i][1][k], c[i][2][k], u[1]);
  if constexpr (D == 3) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) fwd(c[i][j][0], c[i][j][1], c[i][j][2], u[2]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) c[i][j][k] *= inv;
  const double om = (double)p.om, omb = (double)p.om_b;
  const double h3 = 1.0 - (double)p.hi[0], h4 = 1.0 - (double)p.hi[1];
  const double h5 = 1.0 - (double)p.hi[2], h6 = 1.0 - (double)p.hi[3];
  if constexpr (D == 2) {
    const double c20 = c[2][0][0], c02 = c[0][2][0], c11 = c[1][1][0];
    const double k22 = c[2][2][0] - c20 * c02 - 2.0 * c11 * c11;
    // second order: shear (traceless + off-diagonal) and bulk (trace)
    const double tr = 0.5 * (c20 + c02 - 2.0 * cs2);
    const double K20 = cs2 + (1.0 - om) * (c20 - cs2 - tr) + (1.0 - omb) * tr;
    const double K02 = cs2 + (1.0 - om) * (c02 - cs2 - tr) + (1.0 - omb) * tr;
    const double K11 = (1.0 - om) * c11;
    c[2][0][0] = K20;
    c[0][2][0] = K02;
    c[1][1][0] = K11;
    c[2][1][0] *= h3;
    c[1][2][0] *= h3;
    c[2][2][0] = h4 * k22 + K20 * K02 + 2.0 * K11 * K11;
  } else {
    // second-order central moments = cumulants
    const double x2 = c[2][0][0], y2 = c[0][2][0], z2 = c[0][0][2];
    const double xy = c[1][1][0], xz = c[1][0][1], yz = c[0][1][1];
    // third order (= central moments)
    const double x2y = c[2][1][0], x2z = c[2][0][1], xy2 = c[1][2][0], y2z = c[0][2][1], xz2 = c[1][0][2],
                 yz2 = c[0][1][2], xyz = c[1][1][1];
    // fourth order cumulants
    const double k220 = c[2][2][0] - x2 * y2 - 2.0 * xy * xy;
    const double k202 = c[2][0][2] - x2 * z2 - 2.0 * xz * xz;
    const double k022 = c[0][2][2] - y2 * z2 - 2.0 * yz * yz;
    const double k211 = c[2][1][1] - x2 * yz - 2.0 * xy * xz;
    const double k121 = c[1][2][1] - y2 * xz - 2.0 * xy * yz;
    const double k112 = c[1][1][2] - z2 * xy - 2.0 * xz * yz;
    // fifth order
    const double k221 = c[2][2][1] - x2 * y2z - y2 * x2z - 4.0 * xy * xyz - 2.0 * xz * xy2 - 2.0 * yz * x2y;
    const double k212 = c[2][1][2] - x2 * yz2 - z2 * x2y - 4.0 * xz * xyz - 2.0 * xy * xz2 - 2.0 * yz * x2z;
    const double k122 = c[1][2][2] - y2 * xz2 - z2 * xy2 - 4.0 * yz * xyz - 2.0 * xy * yz2 - 2.0 * xz * y2z;
    // sixth order
    const double k222 = c[2][2][2] -
                        (x2 * c[0][2][2] + y2 * c[2][0][2] + z2 * c[2][2][0] + 4.0 * xy * c[1][1][2] +
                         4.0 * xz * c[1][2][1] + 4.0 * yz * c[2][1][1]) -
                        (2.0 * x2y * yz2 + 2.0 * x2z * y2z + 2.0 * xy2 * xz2 + 4.0 * xyz * xyz) +
                        2.0 * (x2 * y2 * z2 + 2.0 * x2 * yz * yz + 2.0 * y2 * xz * xz + 2.0 * z2 * xy * xy +
                               8.0 * xy * xz * yz);
    // relax
    const double tr = (x2 + y2 + z2 - 3.0 * cs2) / 3.0;
    const double X2 = cs2 + (1.0 - om) * (x2 - cs2 - tr) + (1.0 - omb) * tr;
    const double Y2 = cs2 + (1.0 - om) * (y2 - cs2 - tr) + (1.0 - omb) * tr;
    const double Z2 = cs2 + (1.0 - om) * (z2 - cs2 - tr) + (1.0 - omb) * tr;
    const double XY = (1.0 - om) * xy, XZ = (1.0 - om) * xz, YZ = (1.0 - om) * yz;
    const double X2Y = h3 * x2y, X2Z = h3 * x2z, XY2 = h3 * xy2, Y2Z = h3 * y2z, XZ2 = h3 * xz2, YZ2 = h3 * yz2,
                 XYZ = h3 * xyz;
    const double K220 = h4 * k220, K202 = h4 * k202, K022 = h4 * k022, K211 = h4 * k211, K121 = h4 * k121,
                 K112 = h4 * k112;
    const double K221 = h5 * k221, K212 = h5 * k212, K122 = h5 * k122, K222 = h6 * k222;
    // back to central moments
    c[2][0][0] = X2;
    c[0][2][0] = Y2;
    c[0][0][2] = Z2;
    c[1][1][0] = XY;
    c[1][0][1] = XZ;
    c[0][1][1] = YZ;
    c[2][1][0] = X2Y;
    c[2][0][1] = X2Z;
    c[1][2][0] = XY2;
    c[0][2][1] = Y2Z;
    c[1][0][2] = XZ2;
    c[0][1][2] = YZ2;
    c[1][1][1] = XYZ;
    const double C220 = K220 + X2 * Y2 + 2.0 * XY * XY;
    const double C202 = K202 + X2 * Z2 + 2.0 * XZ * XZ;
    const double C022 = K022 + Y2 * Z2 + 2.0 * YZ * YZ;
    const double C211 = K211 + X2 * YZ + 2.0 * XY * XZ;
    const double C121 = K121 + Y2 * XZ + 2.0 * XY * YZ;
    const double C112 = K112 + Z2 * XY + 2.0 * XZ * YZ;
    c[2][2][0] = C220;
    c[2][0][2] = C202;
    c[0][2][2] = C022;
    c[2][1][1] = C211;
    c[1][2][1] = C121;
    c[1][1][2] = C112;
    c[2][2][1] = K221 + X2 * Y2Z + Y2 * X2Z + 4.0 * XY * XYZ + 2.0 * XZ * XY2 + 2.0 * YZ * X2Y;
    c[2][1][2] = K212 + X2 * YZ2 + Z2 * X2Y + 4.0 * XZ * XYZ + 2.0 * XY * XZ2 + 2.0 * YZ * X2Z;
    c[1][2][2] = K122 + Y2 * XZ2 + Z2 * XY2 + 4.0 * YZ * XYZ + 2.0 * XY * YZ2 + 2.0 * XZ * Y2Z;
    // sixth order: partitions {6}, {2,4}, {3,3}, {2,2,2}, expressed with the
    // relaxed cumulants of orders 2..4
    c[2][2][2] = K222 +
                 (X2 * K022 + Y2 * K202 + Z2 * K220 + 4.0 * XY * K112 + 4.0 * XZ * K121 + 4.0 * YZ * K211) +
                 (2.0 * X2Y * YZ2 + 2.0 * X2Z * Y2Z + 2.0 * XY2 * XZ2 + 4.0 * XYZ * XYZ) +
                 (X2 * Y2 * Z2 + 2.0 * X2 * YZ * YZ + 2.0 * Y2 * XZ * XZ + 2.0 * Z2 * XY * XY + 8.0 * XY * XZ * YZ);
  }
  // back-transforms with the mean velocity, then scale by rho
  auto bwd = [](double& a, double& b, double& e, double v) {
    const double k0 = a, k1 = b, k2 = e, v2 = v * v;
    a = 0.5 * (k0 * (v2 - v) + k1 * (2.0 * v - 1.0) + k2);
    b = k0 * (1.0 - v2) - 2.0 * v * k1 - k2;
    e = 0.5 * (k0 * (v2 + v) + k1 * (2.0 * v + 1.0) + k2);
  };
  if constexpr (D == 3) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) bwd(c[i][j][0], c[i][j][1], c[i][j][2], u[2]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < NK; ++k) bwd(c[i][0][k], c[i][1][k], c[i][2][k], u[1]);
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < NK; ++k) bwd(c[0][j][k], c[1][j][k], c[2][j][k], u[0]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int q = qindex<L>(i - 1, j - 1, D == 3 ? k - 1 : 0);
        f[q] = R(rho * c[i][j][k] - weight<L>(q) * rho0);
      }
}

// ---------------------------------------------------------------- KBC
// Entropic KBC-type collision (Sec. III-C "Entropic KBC Models"): an MRT
// method in the lattice-weighted basis whose second-order moments relax with
// fixed rates (shear omega, bulk omega_b) and whose moments of order >= 3
// relax with one rate omega_h chosen per cell, from the entropy condition
// with ln x ~ x - 1:
//   omega_h = 1 + [(1 - omega) <ds, dh>_E + (1 - omega_b) <db, dh>_E] / <dh, dh>_E,
//   <a, b>_E = sum_q a_q b_q / f^eq_q,
// (the paper's closed form for omega_b = omega), omega_h = 1 if dh = 0.
// The parts of the non-equilibrium n = f - f^eq are obtained in population
// space without a moment basis: the second-order part is the Hermite
// projection w_q H2(c_q):Pi / (2 c_s^4), H2 = c c - c_s^2 I, Pi = sum c c n
// (the weighted basis spans the same order-2 space on all three stencils);
// its bulk part is w_q (|c|^2 - D c_s^2) tr Pi / (2 D c_s^4); the first-order
// part (Guo's half-force shift) is w_q c_q . J / c_s^2, J = sum c n; the rest
// of n is dh.  The Guo source has components of orders 1 and 2 only and
// enters as in the MRT operator, (1 - omega/2) on its shear and
// (1 - omega_b/2) on its bulk part.
// Reciprocal for the entropic weights 1/f^eq, which only set the rate
// omega_h: in FP32 the hardware reciprocal (1 ulp); in FP64 the hardware
// approximation refined by two Newton steps r <- r (2 - x r).
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  return r * (2.0 - x * r);
}

template <class L, class R>
__device__ __forceinline__ void collide_kbc(R* f, const R* F, const CollideParams<R>& p) {
  // Every quantity is split over the (q, opp q) pairs: f^eq, the order-2
  // parts and the source's order-2 part are even in c, the order-1 parts
  // odd, so each pair costs one evaluation of each.
  constexpr int D = L::DIM, H = L::H;
  constexpr R cs2 = R(1.0 / 3.0);
  R drho = f[0], jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    const R sp = f[q] + f[q + H], dm = f[q] - f[q + H];
    drho += sp;
    if (L::c(q, 0) != 0) jx += R(L::c(q, 0)) * dm;
    if (L::c(q, 1) != 0) jy += R(L::c(q, 1)) * dm;
    if (L::c(q, 2) != 0) jz += R(L::c(q, 2)) * dm;
  }
  const R rho = p.rho0 + drho;
  const R rr = p.compressible ? rho : p.rho0;
  const R inv = R(1) / rr;
  const R ux = (jx + R(0.5) * F[0]) * inv, uy = (jy + R(0.5) * F[1]) * inv,
          uz = (jz + R(0.5) * F[2]) * inv;
  const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R uF = ux * F[0] + uy * F[1] + uz * F[2];
  // pass 1: non-equilibrium n = f - f^eq (f^eq = f - n later) and its moments
  R n[L::Q];
  n[0] = f[0] - R(weight<L>(0)) * (drho - rr * usq);
  R Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0, Jx = 0, Jy = 0, Jz = 0;
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    const int o = q + H;
    const R w = R(weight<L>(q));
    const R cu = cdot<L>(q, ux, uy, uz);
    const R E = w * (drho + rr * (R(4.5) * cu * cu - usq));   // f^eq shifted by w rho_0: E +- O
    const R O = w * rr * R(3) * cu;
    n[q] = f[q] - (E + O);
    n[o] = f[o] - (E - O);
    const R sp = n[q] + n[o], dm = n[q] - n[o];
    const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
    if (cx != 0) { Pxx += sp; Jx += R(cx) * dm; }
    if (cy != 0) { Pyy += sp; Jy += R(cy) * dm; }
    if (cz != 0) { Pzz += sp; Jz += R(cz) * dm; }
    if (cx * cy != 0) Pxy += R(cx * cy) * sp;
    if (cx * cz != 0) Pxz += R(cx * cz) * sp;
    if (cy * cz != 0) Pyz += R(cy * cz) * sp;
  }
  const R tr = Pxx + Pyy + Pzz;
  const R trD = tr * (R(1) / R(D));
  // second-order part of n at q (Hermite projection, even in c), its bulk part
  auto d2_of = [&](int q) {
    const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
    R h2 = -cs2 * tr;
    if (cx != 0) h2 += Pxx;
    if (cy != 0) h2 += Pyy;
    if (cz != 0) h2 += Pzz;
    if (cx * cy != 0) h2 += R(2 * cx * cy) * Pxy;
    if (cx * cz != 0) h2 += R(2 * cx * cz) * Pxz;
    if (cy * cz != 0) h2 += R(2 * cy * cz) * Pyz;
    return R(4.5 * weight<L>(q)) * h2;
  };
  auto db_of = [&](int q) {
    const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
    return R(4.5 * weight<L>(q) * ((double)(cx * cx + cy * cy + cz * cz) - D / 3.0)) * trD;
  };
  // pass 2: dh (kept in n) and the entropic products
  R sh = 0, bh = 0, hh = 0;
  {
    const R d2 = d2_of(0), db = db_of(0);   // the rest population has no shear part: d2 = db
    const R dh = n[0] - d2;
    const R dhe = dh * recip(R(weight<L>(0)) * p.rho0 + (f[0] - n[0]));
    bh += db * dhe;
    hh += dh * dhe;
    n[0] = dh;
  }
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    const int o = q + H;
    const R d2 = d2_of(q), db = db_of(q);
    const R cJ = R(3 * weight<L>(q)) * cdot<L>(q, Jx, Jy, Jz);
    const R dq = n[q] - d2 - cJ, dp = n[o] - d2 + cJ;
    const R eq = dq * recip(R(weight<L>(q)) * p.rho0 + (f[q] - n[q]));
    const R ep = dp * recip(R(weight<L>(q)) * p.rho0 + (f[o] - n[o]));
    sh += (d2 - db) * (eq + ep);
    bh += db * (eq + ep);
    hh += dq * eq + dp * ep;
    n[q] = dq;
    n[o] = dp;
  }
  const R om = p.om, omb = p.om_b;
  const R omh = hh > R(0) ? R(1) + ((R(1) - om) * sh + (R(1) - omb) * bh) / hh : R(1);
  const R fs = R(1) - R(0.5) * om, fbs = (R(1) - R(0.5) * omb) - fs;
  const R dom = om - omb;
  const R uFD = R(2) * uF * (R(1) / R(D));   // trace of the source's second moment u F + F u, over D
  // pass 3: relax; the Guo source's order-1 part (odd) enters fully, its
  // order-2 part (even) with (1 - omega/2) (shear) and (1 - omega_b/2) (bulk)
  auto s2b_of = [&](int q) {
    const int cx = L::c(q, 0), cy = L::c(q, 1), cz = L::c(q, 2);
    return R(4.5 * weight<L>(q) * ((double)(cx * cx + cy * cy + cz * cz) - D / 3.0)) * uFD;
  };
  f[0] = f[0] - om * d2_of(0) + dom * db_of(0) - omh * n[0] + fs * (R(-3 * weight<L>(0)) * uF) +
         fbs * s2b_of(0);
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    const int o = q + H;
    const R w = R(weight<L>(q));
    const R cu = cdot<L>(q, ux, uy, uz);
    const R cF = cdot<L>(q, F[0], F[1], F[2]);
    const R even = -om * d2_of(q) + dom * db_of(q) + fs * (w * (R(9) * cu * cF - R(3) * uF)) + fbs * s2b_of(q);
    const R odd = R(3) * w * cF;
    f[q] = f[q] + even - omh * n[q] + odd;
    f[o] = f[o] + even - omh * n[o] - odd;
  }
}

template <class L, int M, class R>
__device__ __forceinline__ void collide(R* f, const R* F, const CollideParams<R>& p) {
  if constexpr (M == M_SRT) collide_srt<L>(f, F, p);
  else if constexpr (M == M_SRT_SMAG) collide_srt<L, R, true>(f, F, p);
  else if constexpr (M == M_TRT) collide_trt<L>(f, F, p);
  else if constexpr (M == M_MRT && L::Q == 19) collide_mrt_gs<L>(f, F, p);
  else if constexpr (M == M_MRT) collide_mrt<L>(f, F, p);
  else if constexpr (M == M_MRT_UNIT) collide_mrt_unit<L>(f, F, p);
  else if constexpr (M == M_MRT_SMAG && L::Q == 19) collide_mrt_gs<L, R, true>(f, F, p);
  else if constexpr (M == M_MRT_SMAG) collide_mrt<L, R, true>(f, F, p);
  else if constexpr (M == M_CUMULANT_GEN) collide_cumulant_general<L>(f, F, p);
  else if constexpr (M == M_KBC) collide_kbc<L>(f, F, p);
  else collide_cumulant<L>(f, F, p);
}

}  // namespace lbm
