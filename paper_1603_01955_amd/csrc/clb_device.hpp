// Device-side building blocks of the D2Q9 cascaded LB step for gfx950.
//
// Method: Liu & He, arXiv:1603.01955, Section 2.  All arithmetic is FP64.
// These functions work on one node's nine populations in registers; the
// memory layout belongs to the callers.  Direction order as in Eq. (1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clb {

// Relaxation rates used by one node (Eq. 14, Section 3): s3 (bulk),
// s4 = s5 = s_nu (shear, Eq. 18), s6 = s7 = s_q (Eq. 21), s8.
struct Rates {
  double s3, snu, sq, s8;
};

// ---------------------------------------------------------------------------
// Cascaded collision with semi-implicit forcing, in place on f[9].
//
// The collision of Eqs. (6)-(9) relaxes the central moments of the
// pre-collision f-bar (Eq. 8), taken about the velocity of Eq. (13)
// (rho u = sum e f + rho F / 2, F = (gx, gy) the body acceleration), towards
// those of the equilibrium of Eq. (11): the second-order trace towards
// 2 rho / 3 at s3, the deviator and the shear moment towards 0 at s_nu
// (Eq. 18), the third-order moments towards 0 at s_q (Eq. 21), the
// fourth-order one towards rho / 9 at s8; the force source of Eq. (9) adds
// rho F to the first-order central moments (from -rho F/2 to +rho F/2) and
// nothing above first order.  Here the central moments are reached without
// the moment matrices of Eq. (10): the D2Q9 velocities factor into x and y
// components in {-1, 0, 1}, so a pass along x over each of the three rows
// (moments 1, e_x - u_x, (e_x - u_x)^2 of each row), then a pass along y over
// the three results gives all nine central moments; after the relaxation the
// two passes run backwards (central -> raw -> populations along y, then
// along x).  About 120 FP64 operations instead of the ~220 of the raw-moment
// form of Eqs. (6)-(9) written out.
// THIRD adds (1 - s_q/2) rho F/3 to the post-collision raw moments k_xxy
// (F_y) and k_xyy (F_x): the third-order moments of a second-order
// (Guo-type) force term, which Eq. (9) leaves out; with them Eq. (21)'s
// printed denominator reproduces the slip law of Eq. (19) in a force-driven
// channel.
// ---------------------------------------------------------------------------
namespace detail {

// One axis, forward: populations (m, z, p) at e = -1, 0, +1 -> moments
// (sum, central first, central second) about u, with u2 = u^2, tu = 2u.
__device__ __forceinline__ void axis_central(double m, double z, double p, double u, double u2, double tu,
                                             double& k0, double& k1, double& k2) {
#pragma clang fp contract(off)
  const double sum = p + m, dif = p - m;
  k0 = z + sum;
  k1 = fma(-u, k0, dif);
  k2 = fma(u2, k0, fma(-tu, dif, sum));
}

// One axis, backward: central moments (k0, k1, k2) about u -> populations
// (m, z, p) at e = -1, 0, +1.
__device__ __forceinline__ void axis_populations(double k0, double k1, double k2, double u, double u2, double tu,
                                                 double& m, double& z, double& p) {
#pragma clang fp contract(off)
  const double r1 = fma(u, k0, k1);                   // raw sum of e f
  const double r2 = fma(u2, k0, fma(tu, k1, k2));     // raw sum of e^2 f
  const double h1 = 0.5 * r1;
  z = k0 - r2;
  p = fma(0.5, r2, h1);
  m = fma(0.5, r2, -h1);
}

}  // namespace detail

template <bool FORCE, bool THIRD = false>
__device__ __forceinline__ void collide(double f[9], double gx, double gy, const Rates& s) {
  // Products and sums round on their own except where written as fma(): the
  // same FP64 result in every kernel that inlines this, whatever the
  // compiler fuses around it.
#pragma clang fp contract(off)
  using detail::axis_central;
  using detail::axis_populations;
  // Rows of the velocity set (Eq. 1), each ordered e_x = -1, 0, +1:
  // e_y = 0: f3 f0 f1, e_y = +1: f6 f2 f5, e_y = -1: f7 f4 f8.
  // Zeroth x moment and the moving-population difference of each row.
  const double kz = f[0] + (f[1] + f[3]), tz = f[1] - f[3];
  const double kp = f[2] + (f[5] + f[6]), tp = f[5] - f[6];
  const double km = f[4] + (f[8] + f[7]), tm = f[8] - f[7];
  // Eqs. (12)-(13)
  const double rho = kz + (kp + km);
  const double jx = tz + (tp + tm);
  const double inv_rho = 1.0 / rho;
  const double ux = FORCE ? fma(jx, inv_rho, 0.5 * gx) : jx * inv_rho;
  const double uy = FORCE ? fma(kp - km, inv_rho, 0.5 * gy) : (kp - km) * inv_rho;
  const double ux2 = ux * ux, uy2 = uy * uy, tux = ux + ux, tuy = uy + uy;

  // x pass: central moments along x of each row (order 0 is kz, kp, km).
  double az, bz, cz, ap, bp, cp, am, bm, cm;
  axis_central(f[3], f[0], f[1], ux, ux2, tux, az, bz, cz);
  axis_central(f[6], f[2], f[5], ux, ux2, tux, ap, bp, cp);
  axis_central(f[7], f[4], f[8], ux, ux2, tux, am, bm, cm);
  // y pass: k_ab = central moment of order a in x and b in y.
  double k00, k01, k02, k10, k11, k12, k20, k21, k22;
  axis_central(am, az, ap, uy, uy2, tuy, k00, k01, k02);
  axis_central(bm, bz, bp, uy, uy2, tuy, k10, k11, k12);
  axis_central(cm, cz, cp, uy, uy2, tuy, k20, k21, k22);

  // Relaxation (Eq. 14 rates) and the force source of Eq. (9).
  if (FORCE) {
    k10 = fma(rho, gx, k10);
    k01 = fma(rho, gy, k01);
  }
  const double tr = k20 + k02, dv = k20 - k02;
  const double tr1 = fma(-s.s3, fma(-(2.0 / 3.0), rho, tr), tr);
  const double onu = 1.0 - s.snu, oq = 1.0 - s.sq;
  const double dv1 = onu * dv;
  k20 = 0.5 * (tr1 + dv1);
  k02 = 0.5 * (tr1 - dv1);
  k11 = onu * k11;
  k21 = oq * k21;
  k12 = oq * k12;
  k22 = fma(-s.s8, fma(-(1.0 / 9.0), rho, k22), k22);

  // Back: y pass for each x order, then x pass for each row.
  axis_populations(rho, k01, k02, uy, uy2, tuy, am, az, ap);
  axis_populations(k10, k11, k12, uy, uy2, tuy, bm, bz, bp);
  axis_populations(k20, k21, k22, uy, uy2, tuy, cm, cz, cp);
  axis_populations(az, bz, cz, ux, ux2, tux, f[3], f[0], f[1]);
  axis_populations(ap, bp, cp, ux, ux2, tux, f[6], f[2], f[5]);
  axis_populations(am, bm, cm, ux, ux2, tux, f[7], f[4], f[8]);

  if (FORCE && THIRD) {
    // (1 - s_q/2) rho F / 3 added to the raw moments k_xxy (F_y) and k_xyy
    // (F_x), mapped to populations by the inverse of Eq. (10).
    const double c = (1.0 - 0.5 * s.sq) * (1.0 / 3.0) * rho;
    const double dxxy = c * gy, dxyy = c * gx;
    const double qa = 0.25 * (dxxy + dxyy), qb = 0.25 * (dxxy - dxyy);
    const double hx = 0.5 * dxyy, hy = 0.5 * dxxy;
    f[5] += qa;
    f[7] -= qa;
    f[6] += qb;
    f[8] -= qb;
    f[1] -= hx;
    f[3] += hx;
    f[2] -= hy;
    f[4] += hy;
  }
}

// Equilibrium of Eq. (11).  Its T-moments factor per axis into the D1Q3
// moments (1, u, 1/3 + u^2), so f_i^eq = rho * w(e_ix, ux) * w(e_iy, uy) with
// w(0, u) = 2/3 - u^2 and w(+-1, u) = (1/3 + u^2 +- u) / 2.
__device__ __forceinline__ void equilibrium(double rho, double ux, double uy, double e[9]) {
#pragma clang fp contract(off)
  const double ax0 = 2.0 / 3.0 - ux * ux, axp = 0.5 * (1.0 / 3.0 + ux * ux + ux),
               axm = 0.5 * (1.0 / 3.0 + ux * ux - ux);
  const double ay0 = 2.0 / 3.0 - uy * uy, ayp = 0.5 * (1.0 / 3.0 + uy * uy + uy),
               aym = 0.5 * (1.0 / 3.0 + uy * uy - uy);
  e[0] = rho * ax0 * ay0;
  e[1] = rho * axp * ay0;
  e[2] = rho * ax0 * ayp;
  e[3] = rho * axm * ay0;
  e[4] = rho * ax0 * aym;
  e[5] = rho * axp * ayp;
  e[6] = rho * axm * ayp;
  e[7] = rho * axm * aym;
  e[8] = rho * axp * aym;
}

__device__ __forceinline__ double sum9(const double f[9]) {
#pragma clang fp contract(off)
  return f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
}

// Relaxation rates of a column of the pressure-driven channel from its
// centre-line density rc (Section 3.2): Kn = Kn_out rho_out / rho_c,
// tt = s_nu^-1 - 1/2 = c_tau Kn / (1 + a Kn) with c_tau = sqrt(6/pi) N
// (Eq. 18), s_q^-1 = 1/2 + (3 + 4 pi tt^2 A2) / (D tt) (Eq. 21).
__device__ __forceinline__ void local_rates(double kn_out, double rho_out, double rc, double c_tau, double a,
                                            double A2, double D, double& snu, double& sq, double& kn,
                                            double& tt) {
#pragma clang fp contract(off)
  kn = kn_out * rho_out / rc;
  tt = c_tau * kn / (1.0 + a * kn);
  snu = 1.0 / (0.5 + tt);
  sq = 1.0 / (0.5 + (3.0 + 4.0 * M_PI * tt * tt * A2) / (D * tt));
}

__device__ __forceinline__ void local_rates(double kn_out, double rho_out, double rc, double c_tau, double a,
                                            double A2, double D, double& snu, double& sq) {
  double kn, tt;
  local_rates(kn_out, rho_out, rc, c_tau, a, A2, D, snu, sq, kn, tt);
}

// Density and velocity of a population vector without force (Eqs. 12-13).
__device__ __forceinline__ void rho_u(const double f[9], double& rho, double& ux, double& uy) {
#pragma clang fp contract(off)
  rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  const double inv = 1.0 / rho;
  ux = ((f[1] - f[3]) + (f[5] - f[7]) + (f[8] - f[6])) * inv;
  uy = ((f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8])) * inv;
}

// Sum over the 64 lanes of a wavefront in a fixed order: a butterfly over
// lane distances 32, 16, ..., 1 (cross-lane moves, no LDS, no barrier).  At
// every level lanes i and i ^ d add the same two partial sums, so every lane
// ends with the same bits, and the result does not depend on timing.
__device__ __forceinline__ double wave_sum(double v) {
#pragma clang fp contract(off)
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// SplitMix64 finaliser (Steele, Lea & Flood 2014): first output of a stream
// whose state is `key`.
__device__ __forceinline__ uint64_t splitmix64_first(uint64_t key) {
  uint64_t z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace clb
