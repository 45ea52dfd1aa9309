// Hand-written reverse-mode derivatives of the force-free cascaded collision
// and of the pressure ghost column (device code).
//
// Method: Liu & He, arXiv:1603.01955, Eqs. (6)-(8), (12)-(13) (collision with
// F = 0, the pressure-driven case of Section 3.2) and the equilibrium of
// Eq. (11).  Each function recomputes the forward intermediates from its
// inputs and then propagates adjoints through them in reverse order.
#pragma once

#include "clb_device.hpp"

namespace clb {

// Given the pre-collision populations f and the adjoint lo of the
// post-collision populations, return lf = (d post / d f)^T lo and the
// sensitivities d(lo . post)/d s_nu and d(lo . post)/d s_q (s3, s8 fixed).
__device__ __forceinline__ void collide_vjp(const double f[9], const double lo[9], const Rates& s,
                                            double lf[9], double& l_snu, double& l_sq) {
#pragma clang fp contract(off)
  // ---- forward recompute (Eq. 8, Eq. 13 with F = 0, Eq. 7) ----
  const double f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3], f4 = f[4];
  const double f5 = f[5], f6 = f[6], f7 = f[7], f8 = f[8];
  const double d57 = f5 + f7, d68 = f6 + f8;
  const double diag = d57 + d68;
  const double k_xx = f1 + f3 + diag;
  const double k_yy = f2 + f4 + diag;
  const double k_xy = d57 - d68;
  const double k_xxy = (f5 + f6) - (f7 + f8);
  const double k_xyy = (f5 + f8) - (f6 + f7);
  const double rho = f0 + (f1 + f3) + (f2 + f4) + diag;
  const double jx = (f1 - f3) + (f5 - f7) + (f8 - f6);
  const double jy = (f2 - f4) + (f5 - f7) + (f6 - f8);
  const double inv = 1.0 / rho;
  const double ux = jx * inv, uy = jy * inv;
  const double ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
  const double c3 = (2.0 / 3.0) * rho + rho * (ux2 + uy2) - (k_xx + k_yy);
  const double c4 = rho * (ux2 - uy2) - (k_xx - k_yy);
  const double c5 = rho * uxy - k_xy;
  const double c6 = 2.0 * rho * ux2 * uy + k_xxy - 2.0 * ux * k_xy - uy * k_xx;
  const double c7 = 2.0 * rho * ux * uy2 + k_xyy - 2.0 * uy * k_xy - ux * k_yy;
  // (c8 itself is not needed: g8 enters the outputs linearly)
  const double g3 = s.s3 * (1.0 / 12.0) * c3;
  const double g4 = 0.25 * s.snu * c4;
  const double g5 = 0.25 * s.snu * c5;
  const double a34 = 3.0 * g3 + g4;
  const double b34 = 3.0 * g3 - g4;
  const double g6 = 0.25 * s.sq * c6 - 0.5 * uy * a34 - 2.0 * ux * g5;
  const double g7 = 0.25 * s.sq * c7 - 0.5 * ux * b34 - 2.0 * uy * g5;

  // ---- reverse: outputs of Eq. (6) ----
  const double lt = lo[5] + lo[6] + lo[7] + lo[8];      // t = 2 g3 + g8
  double lg3 = -4.0 * lo[0] - lo[1] - lo[2] - lo[3] - lo[4] + 2.0 * lt;
  double lg4 = lo[1] - lo[2] + lo[3] - lo[4];
  double lg5 = lo[5] - lo[6] + lo[7] - lo[8];
  double lg6 = 2.0 * lo[2] - 2.0 * lo[4] - lo[5] - lo[6] + lo[7] + lo[8];
  double lg7 = 2.0 * lo[1] - 2.0 * lo[3] - lo[5] + lo[6] + lo[7] - lo[8];
  const double lg8 = 4.0 * lo[0] - 2.0 * (lo[1] + lo[2] + lo[3] + lo[4]) + lt;

  // g8 = s8/4 c8 - 2 g3 - 1/2 uy2 a34 - 1/2 ux2 b34 - 4 uxy g5 - 2 uy g6 - 2 ux g7
  double lc8 = 0.25 * s.s8 * lg8;
  lg3 += -2.0 * lg8;
  double luy2 = -0.5 * a34 * lg8;
  double la34 = -0.5 * uy2 * lg8;
  double lux2 = -0.5 * b34 * lg8;
  double lb34 = -0.5 * ux2 * lg8;
  double luxy = -4.0 * g5 * lg8;
  lg5 += -4.0 * uxy * lg8;
  double luy = -2.0 * g6 * lg8;
  lg6 += -2.0 * uy * lg8;
  double lux = -2.0 * g7 * lg8;
  lg7 += -2.0 * ux * lg8;

  // g7 = sq/4 c7 - 1/2 ux b34 - 2 uy g5
  const double lc7 = 0.25 * s.sq * lg7;
  l_sq = 0.25 * c7 * lg7;
  lux += -0.5 * b34 * lg7;
  lb34 += -0.5 * ux * lg7;
  luy += -2.0 * g5 * lg7;
  lg5 += -2.0 * uy * lg7;

  // g6 = sq/4 c6 - 1/2 uy a34 - 2 ux g5
  const double lc6 = 0.25 * s.sq * lg6;
  l_sq += 0.25 * c6 * lg6;
  luy += -0.5 * a34 * lg6;
  la34 += -0.5 * uy * lg6;
  lux += -2.0 * g5 * lg6;
  lg5 += -2.0 * ux * lg6;

  // a34 = 3 g3 + g4, b34 = 3 g3 - g4
  lg3 += 3.0 * (la34 + lb34);
  lg4 += la34 - lb34;

  // g5 = s_nu/4 c5, g4 = s_nu/4 c4, g3 = s3/12 c3
  const double lc5 = 0.25 * s.snu * lg5;
  const double lc4 = 0.25 * s.snu * lg4;
  l_snu = 0.25 * (c5 * lg5 + c4 * lg4);
  const double lc3 = s.s3 * (1.0 / 12.0) * lg3;

  // ---- reverse: the c's (Eq. 7) ----
  double lrho = 0.0, lkxx = 0.0, lkyy = 0.0, lkxy = 0.0, lkxxy = 0.0, lkxyy = 0.0, ldiag = 0.0;
  // c8
  lrho += (1.0 / 9.0 + 3.0 * ux2 * uy2) * lc8;
  lux2 += (3.0 * rho * uy2 - k_yy) * lc8;
  luy2 += (3.0 * rho * ux2 - k_xx) * lc8;
  ldiag += -lc8;
  lux += 2.0 * k_xyy * lc8;
  lkxyy += 2.0 * ux * lc8;
  luy += 2.0 * k_xxy * lc8;
  lkxxy += 2.0 * uy * lc8;
  lkyy += -ux2 * lc8;
  lkxx += -uy2 * lc8;
  luxy += -4.0 * k_xy * lc8;
  lkxy += -4.0 * uxy * lc8;
  // c7
  lrho += 2.0 * ux * uy2 * lc7;
  lux += (2.0 * rho * uy2 - k_yy) * lc7;
  luy2 += 2.0 * rho * ux * lc7;
  lkxyy += lc7;
  luy += -2.0 * k_xy * lc7;
  lkxy += -2.0 * uy * lc7;
  lkyy += -ux * lc7;
  // c6
  lrho += 2.0 * ux2 * uy * lc6;
  lux2 += 2.0 * rho * uy * lc6;
  luy += (2.0 * rho * ux2 - k_xx) * lc6;
  lkxxy += lc6;
  lux += -2.0 * k_xy * lc6;
  lkxy += -2.0 * ux * lc6;
  lkxx += -uy * lc6;
  // c5
  lrho += uxy * lc5;
  luxy += rho * lc5;
  lkxy += -lc5;
  // c4
  lrho += (ux2 - uy2) * lc4;
  lux2 += rho * lc4;
  luy2 += -rho * lc4;
  lkxx += -lc4;
  lkyy += lc4;
  // c3
  lrho += (2.0 / 3.0 + ux2 + uy2) * lc3;
  lux2 += rho * lc3;
  luy2 += rho * lc3;
  lkxx += -lc3;
  lkyy += -lc3;

  // ---- reverse: velocity (Eq. 13) ----
  lux += 2.0 * ux * lux2 + uy * luxy;
  luy += 2.0 * uy * luy2 + ux * luxy;
  const double ljx = inv * lux;
  const double ljy = inv * luy;
  lrho += -inv * (ux * lux + uy * luy);   // d(j/rho)/d rho = -u/rho

  // ---- reverse: raw moments (Eq. 8) ----
  ldiag += lkxx + lkyy + lrho;
  const double ld57 = ldiag + lkxy;
  const double ld68 = ldiag - lkxy;
  lf[0] = lo[0] + lrho;
  lf[1] = lo[1] + lkxx + lrho + ljx;
  lf[2] = lo[2] + lkyy + lrho + ljy;
  lf[3] = lo[3] + lkxx + lrho - ljx;
  lf[4] = lo[4] + lkyy + lrho - ljy;
  lf[5] = lo[5] + ld57 + lkxxy + lkxyy + ljx + ljy;
  lf[6] = lo[6] + ld68 + lkxxy - lkxyy - ljx + ljy;
  lf[7] = lo[7] + ld57 - lkxxy - lkxyy - ljx - ljy;
  lf[8] = lo[8] + ld68 - lkxxy + lkxyy + ljx - ljy;
}

// Per-axis factor of the equilibrium (Eq. 11) and its derivative in u:
// w(0, u) = 2/3 - u^2, w(+-1, u) = (1/3 + u^2 +- u) / 2.
__device__ __forceinline__ double eq_w(int e, double u) {
#pragma clang fp contract(off)
  return e == 0 ? 2.0 / 3.0 - u * u : 0.5 * (1.0 / 3.0 + u * u + (double)e * u);
}
__device__ __forceinline__ double eq_dw(int e, double u) {
#pragma clang fp contract(off)
  return e == 0 ? -2.0 * u : u + 0.5 * (double)e;
}

__device__ __forceinline__ int ex_of(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__device__ __forceinline__ int ey_of(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}

// Reverse of the pressure ghost column of one row (the extrapolation used by
// the forward gather): g = f^eq(2 rho_b - rho_1, 2 u_1 - u_2) + f_1 - f^eq(rho_1, u_1)
// with (rho_1, u_1) from f1 (adjacent column) and u_2 from f2 (next column).
// Only the directions entering the channel are used downstream (1, 5, 8 at
// the inlet, 3, 6, 7 at the outlet), so lg = dL/dg has those three entries;
// adds dL/df1 to l1 and dL/df2 to l2.
template <bool INLET>
__device__ __forceinline__ void ghost_vjp(const double f1[9], const double f2[9], double rho_b, const double lg[3],
                                          double l1[9], double l2[9]) {
#pragma clang fp contract(off)
  constexpr int dirs[3] = {INLET ? 1 : 3, INLET ? 5 : 6, INLET ? 8 : 7};
  double rho1, ux1, uy1, rho2, ux2, uy2;
  rho_u(f1, rho1, ux1, uy1);
  rho_u(f2, rho2, ux2, uy2);
  const double rhog = 2.0 * rho_b - rho1;
  const double ugx = 2.0 * ux1 - ux2, ugy = 2.0 * uy1 - uy2;
  double l_rhog = 0.0, l_ugx = 0.0, l_ugy = 0.0, l_rho1 = 0.0, l_u1x = 0.0, l_u1y = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = dirs[k];
    const int ex = ex_of(i), ey = ey_of(i);
    const double wgx = eq_w(ex, ugx), wgy = eq_w(ey, ugy);
    const double w1x = eq_w(ex, ux1), w1y = eq_w(ey, uy1);
    l_rhog += lg[k] * (wgx * wgy);
    l_ugx += lg[k] * rhog * (eq_dw(ex, ugx) * wgy);
    l_ugy += lg[k] * rhog * (wgx * eq_dw(ey, ugy));
    l_rho1 -= lg[k] * (w1x * w1y);
    l_u1x -= lg[k] * rho1 * (eq_dw(ex, ux1) * w1y);
    l_u1y -= lg[k] * rho1 * (w1x * eq_dw(ey, uy1));
    l1[i] += lg[k];   // the copied f_1 term
  }
  // rho_g = 2 rho_b - rho_1, u_g = 2 u_1 - u_2
  l_rho1 -= l_rhog;
  l_u1x += 2.0 * l_ugx;
  l_u1y += 2.0 * l_ugy;
  const double l_u2x = -l_ugx, l_u2y = -l_ugy;
  // u = j / rho:  dj = du / rho,  drho = -(u . du) / rho
  const double lj1x = l_u1x / rho1, lj1y = l_u1y / rho1;
  l_rho1 -= (ux1 * l_u1x + uy1 * l_u1y) / rho1;
  const double lj2x = l_u2x / rho2, lj2y = l_u2y / rho2;
  const double l_rho2 = -(ux2 * l_u2x + uy2 * l_u2y) / rho2;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double ex = (double)ex_of(i), ey = (double)ey_of(i);
    l1[i] += l_rho1 + ex * lj1x + ey * lj1y;
    l2[i] += l_rho2 + ex * lj2x + ey * lj2y;
  }
}

}  // namespace clb
