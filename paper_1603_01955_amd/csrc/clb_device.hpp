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
// Cascaded collision with semi-implicit forcing, in place on f[9]:
//   raw moments of the pre-collision f-bar (Eq. 8), velocity from Eq. (13)
//   (rho u = sum e f + rho F / 2, F = (gx, gy) the body acceleration),
//   collision kernels g3..g8 in ascending order (Eq. 7, g0 = g1 = g2 = 0),
//   forcing S = T^-1 S_hat (Eqs. 9, 10) with T^-1 in closed form, and the
//   update f + K g + S written out per direction (Eqs. 4, 6).
// THIRD adds (1 - s_q/2) rho F/3 to the source's raw moments k_xxy (F_y) and
// k_xyy (F_x): the third-order moments of a second-order (Guo-type) force
// term, which Eq. (9) leaves out; with them Eq. (21)'s printed denominator
// reproduces the slip law of Eq. (19) in a force-driven channel.
// ---------------------------------------------------------------------------
template <bool FORCE, bool THIRD = false>
__device__ __forceinline__ void collide(double f[9], double gx, double gy, const Rates& s) {
  // Products and sums round on their own except where written as fma(): the
  // same FP64 result in every kernel that inlines this, whatever the
  // compiler fuses around it.
#pragma clang fp contract(off)
  const double f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3], f4 = f[4];
  const double f5 = f[5], f6 = f[6], f7 = f[7], f8 = f[8];

  // Eq. (8)
  const double d57 = f5 + f7, d68 = f6 + f8;
  const double diag = d57 + d68;                      // k'_xxyy
  const double s13 = f1 + f3, s24 = f2 + f4;
  const double k_xx = s13 + diag;
  const double k_yy = s24 + diag;
  const double k_xy = d57 - d68;
  const double k_xxy = (f5 + f6) - (f7 + f8);
  const double k_xyy = (f5 + f8) - (f6 + f7);
  const double rho = f0 + s13 + s24 + diag;
  const double m57 = f5 - f7;
  const double jx = (f1 - f3) + m57 + (f8 - f6);
  const double jy = (f2 - f4) + m57 + (f6 - f8);

  // Eq. (13)
  const double inv_rho = 1.0 / rho;
  const double ux = FORCE ? fma(jx, inv_rho, 0.5 * gx) : jx * inv_rho;
  const double uy = FORCE ? fma(jy, inv_rho, 0.5 * gy) : jy * inv_rho;
  const double ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
  const double tux = 2.0 * ux, tuy = 2.0 * uy, trho = 2.0 * rho;

  // Eq. (7): the force corrections are the "-1/2 rho (...)" terms.
  double c3 = fma(rho, ux2 + uy2, (2.0 / 3.0) * rho) - (k_xx + k_yy);
  double c4 = fma(rho, ux2 - uy2, -(k_xx - k_yy));
  double c5 = fma(rho, uxy, -k_xy);
  double c6 = fma(-uy, k_xx, fma(-tux, k_xy, fma(trho * ux2, uy, k_xxy)));
  double c7 = fma(-ux, k_yy, fma(-tuy, k_xy, fma(trho * uy2, ux, k_xyy)));
  const double inner =
      fma(4.0 * uxy, k_xy, fma(uy2, k_xx, fma(ux2, k_yy, fma(-tuy, k_xxy, fma(-tux, k_xyy, diag)))));
  double c8 = fma(3.0 * rho * ux2, uy2, rho * (1.0 / 9.0)) - inner;
  if (FORCE) {
    c3 -= rho * fma(gx, ux, gy * uy);
    c4 -= rho * fma(gx, ux, -(gy * uy));
    c5 -= 0.5 * rho * fma(gx, uy, gy * ux);
    c6 -= 0.5 * rho * fma(gy, ux2, 2.0 * gx * uxy);
    c7 -= 0.5 * rho * fma(gx, uy2, 2.0 * gy * uxy);
    c8 -= rho * fma(gx * ux, uy2, gy * uy * ux2);
  }
  const double g3 = s.s3 * (1.0 / 12.0) * c3;
  const double qnu = 0.25 * s.snu;
  const double g4 = qnu * c4;
  const double g5 = qnu * c5;
  const double a34 = fma(3.0, g3, g4);    // appears in g6 and g8
  const double b34 = fma(3.0, g3, -g4);   // appears in g7 and g8
  const double qq = 0.25 * s.sq;
  const double g6 = fma(-tux, g5, fma(-0.5 * uy, a34, qq * c6));
  const double g7 = fma(-tuy, g5, fma(-0.5 * ux, b34, qq * c7));
  const double g8 = fma(-tux, g7, fma(-tuy, g6, fma(-4.0 * uxy, g5, fma(-0.5 * ux2, b34,
                    fma(-0.5 * uy2, a34, fma(-2.0, g3, 0.25 * s.s8 * c8))))));

  // Eq. (6): f + K g (columns of K from Eq. 3).
  const double g38 = g3 - g8, g78 = g7 - g8, g68 = g6 - g8;
  double o0 = fma(-4.0, g38, f0);
  double o1 = fma(2.0, g78, (f1 - g3) + g4);
  double o2 = fma(2.0, g68, (f2 - g3) - g4);
  double o3 = fma(-2.0, g7 + g8, (f3 - g3) + g4);
  double o4 = fma(-2.0, g6 + g8, (f4 - g3) - g4);
  const double t = fma(2.0, g3, g8);
  double o5 = f5 + t + g5 - g6 - g7;
  double o6 = f6 + t - g5 - g6 + g7;
  double o7 = f7 + t + g5 + g6 + g7;
  double o8 = f8 + t - g5 + g6 - g7;

  if (FORCE) {
    // Eq. (9) source moments in the basis of Eq. (10) ...
    const double Sx = rho * gx, Sy = rho * gy;
    const double Sxy = rho * fma(ux, gy, uy * gx);
    double Sxxy = fma(Sy, ux2, 2.0 * Sx * uxy);
    double Sxyy = fma(Sx, uy2, 2.0 * Sy * uxy);
    if (THIRD) {
      const double c = (1.0 - 0.5 * s.sq) * (1.0 / 3.0);
      Sxxy = fma(c, Sy, Sxxy);
      Sxyy = fma(c, Sx, Sxyy);
    }
    const double Sxxyy = 2.0 * fma(Sx * ux, uy2, Sy * uy * ux2);
    const double Sxx = 2.0 * Sx * ux;   // (S3 + S4)/2
    const double Syy = 2.0 * Sy * uy;   // (S3 - S4)/2
    // ... mapped back to populations by the inverse of T (closed form).
    o0 += Sxxyy - Sxx - Syy;
    o1 += 0.5 * (Sxx - Sxxyy + Sx - Sxyy);
    o3 += 0.5 * (Sxx - Sxxyy - Sx + Sxyy);
    o2 += 0.5 * (Syy - Sxxyy + Sy - Sxxy);
    o4 += 0.5 * (Syy - Sxxyy - Sy + Sxxy);
    o5 += 0.25 * (Sxxyy + Sxy + Sxxy + Sxyy);
    o6 += 0.25 * (Sxxyy - Sxy + Sxxy - Sxyy);
    o7 += 0.25 * (Sxxyy + Sxy - Sxxy - Sxyy);
    o8 += 0.25 * (Sxxyy - Sxy - Sxxy + Sxyy);
  }
  f[0] = o0; f[1] = o1; f[2] = o2; f[3] = o3; f[4] = o4;
  f[5] = o5; f[6] = o6; f[7] = o7; f[8] = o8;
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

// SplitMix64 finaliser (Steele, Lea & Flood 2014): first output of a stream
// whose state is `key`.
__device__ __forceinline__ uint64_t splitmix64_first(uint64_t key) {
  uint64_t z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace clb
