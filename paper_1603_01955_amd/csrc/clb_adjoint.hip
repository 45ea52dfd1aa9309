// Hand-written adjoint of the pressure-driven CLB run (gfx950).
//
// Method: Liu & He, arXiv:1603.01955, Section 3.2 (long channel, pressure
// inlet/outlet, local Kn(x)), with the step of Eqs. (4)-(8), (13), (18),
// (20), (21).  Loss of a run of T steps from the linear-density start:
//   L = (1/nx) sum_x (dp(x) - dp*(x))^2 + ((m - m*) / m*)^2,
// dp the centre-line pressure deviation and m = sum_y rho u_x at the outlet
// column, both from the pre-collision state at step T.  Parameters: the
// Bosanquet factor a (Eq. 16), the slip coefficients A1 (through r, Eq. 21)
// and A2 = B2 (Eq. 21), and the bounce-back fraction r (Eq. 20).
//
// One step is P' = C(G(P; r); s(x)) with G the gather (streaming, walls,
// ghost columns) and s(x) = (s_nu, s_q) from rho_c(x) of the same gathered
// state.  The reverse step for lambda' = dL/dP':
//   lambda' = G^T lpre' as a pull over the uses of each P'_i(x, y) (regular
//     streaming, the CBBSR mixes, the reverse of the ghost extrapolation at
//     the first two and last two columns), evaluated on the fly;
//   lpre = (dC/dpre)^T lambda' at pre = G(P) per node; per column the rate
//     sensitivities flow through s(tau(Kn(rho_c))) back into lpre at the
//     centre rows and into dL/da, dL/dA2; wall rows add lpre . dpre/dr to
//     dL/dr.
// Both halves run in one kernel per reverse step (k_adj_step).
// The forward run keeps ceil(T/K) checkpoints.  The backward sweep reverses
// the segments of K steps from last to first; each segment is recomputed from
// its checkpoint (with its ghost columns, k_ghosts) on a second stream while
// the segment after it is being reversed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <new>

#include "clb.h"
#include "clb_adjoint_device.hpp"
#include "clb_device.hpp"
#include "clb_gather.hpp"
#include "clb_internal.hpp"
#include "clb_trace.hpp"

namespace clb {
namespace {

// Column blocks of 256 threads: (256 / RY) columns x RY row lanes, RY the
// smallest of 16, 32, 64 covering ny (one node per thread up to ny = 64).
inline int adj_rows(int ny) { return ny <= 16 ? 16 : (ny <= 32 ? 32 : 64); }

struct AdjArgs {
  const double* P;       // state P_n (device layout)
  const double* gh;      // ghost columns of P_n, [2][9][ny] (inlet, outlet)
  const double* Pn1;     // state P_{n+1} (ghost reverse of the pulled adjoint)
  const double* lam;     // lambda_{n+1} (device layout), when not pulled
  const double* lin;     // lpre_{n+1}, pulled through the transposed gather
  double* lpre;          // lpre_n out (device layout); k_adj_gather reads it
  double* out;           // lambda_n (device layout), k_adj_gather
  double* gpart;         // [blocks][3] accumulated (da, dA2, dr)
  Geo g;
  int shift;
  double r;
  double s3, s8;
  double kn, a, A2, tq_den, c_tau;
  double rho_in, rho_out;
  int xcd_remap;         // XCD-aware workgroup order (see logical_block)
};

// lpre . d pre / d r for the wall-replaced entries of node (x, y) (Eq. 20),
// reading the sources again (used off the hot path).
template <class G>
__device__ __forceinline__ double wall_dr(const G& gat, int x, int y, const double lp[9]) {
#pragma clang fp contract(off)
  const int t = gat.v.g.ny - 1;
  const int xsm = gat.shift ? x - 1 : x;
  const int xsp = gat.shift ? x + 1 : x;
  double dr = 0.0;
  if (y == 0) {
    dr += lp[5] * (gat.pop(7, x, 0) - gat.pop(8, xsm, 0));
    dr += lp[6] * (gat.pop(8, x, 0) - gat.pop(7, xsp, 0));
  }
  if (y == t) {
    dr += lp[7] * (gat.pop(5, x, t) - gat.pop(6, xsp, t));
    dr += lp[8] * (gat.pop(6, x, t) - gat.pop(5, xsm, t));
  }
  return dr;
}

// ---------------------------------------------------------------------------
// lambda(x, y) = (G^T lp)(x, y): the adjoint of P_i(x, y) gathered over its
// uses in the gather G(P): regular streaming, the CBBSR mixes of Eq. (20),
// and the reverse of the ghost extrapolation at the first two / last two
// columns (which needs P itself there).  Written branch-free like the forward
// gather: tg_sources selects every address and issues all loads, tg_combine
// does the arithmetic.  XB = 3: x - 1 and x + 1 lie inside the grid; XB = 1:
// any column (uses beyond x = -1 or nx are dropped).
// ---------------------------------------------------------------------------
template <int XB>
__device__ __forceinline__ void tg_sources(const AdjArgs& a, const double* __restrict__ lp, int x, int y, double Lp[9],
                                           double Lq[4]) {
  const int nx = a.g.nx, t = a.g.ny - 1;
  const bool bot = y == 0, top = y == t;
  auto cl = [&](int xx) { return XB == 3 ? xx : (xx < 0 ? 0 : (xx >= nx ? nx - 1 : xx)); };
  auto A = [&](int i, int xx, int yy) { return lp + a.g.index(i, cl(xx), yy); };
  const int ym = bot ? 0 : y - 1, yp = top ? t : y + 1;
  const int xsm = a.shift ? x - 1 : x, xsp = a.shift ? x + 1 : x;
  const double* p[9];
  const double* q[4];
  p[0] = A(0, x, y);
  p[1] = A(1, x + 1, y);
  p[3] = A(3, x - 1, y);
  // directions with e_y = +1 are used at row y + 1, or by the top wall mixes
  p[2] = top ? A(4, x, t) : A(2, x, yp);
  p[5] = top ? A(7, x, t) : A(5, x + 1, yp);
  p[6] = top ? A(8, x, t) : A(6, x - 1, yp);
  // directions with e_y = -1 are used at row y - 1, or by the bottom wall mixes
  p[4] = bot ? A(2, x, 0) : A(4, x, ym);
  p[7] = bot ? A(5, x, 0) : A(7, x - 1, ym);
  p[8] = bot ? A(6, x, 0) : A(8, x + 1, ym);
  // specular uses: pre8(x_s) takes P5(x_s - 1), pre7(x_s) takes P6(x_s + 1),
  // pre6(x_s) takes P7(x_s + 1), pre5(x_s) takes P8(x_s - 1)
  q[0] = top ? A(8, xsp, t) : p[5];
  q[1] = top ? A(7, xsm, t) : p[6];
  q[2] = bot ? A(6, xsm, 0) : p[7];
  q[3] = bot ? A(5, xsp, 0) : p[8];
#pragma unroll
  for (int i = 0; i < 9; ++i) Lp[i] = *p[i];
#pragma unroll
  for (int k = 0; k < 4; ++k) Lq[k] = *q[k];
}

template <int XB>
__device__ __forceinline__ void tg_combine(const AdjArgs& a, int x, int y, const double Lp[9], const double Lq[4],
                                           double out[9]) {
#pragma clang fp contract(off)
  const int nx = a.g.nx, t = a.g.ny - 1;
  const bool bot = y == 0, top = y == t;
  const double r = a.r, omr = 1.0 - a.r;
  auto in = [&](int xx) { return XB == 3 || (xx >= 0 && xx < nx); };
  const int xsm = a.shift ? x - 1 : x, xsp = a.shift ? x + 1 : x;
  out[0] = Lp[0];
  out[1] = in(x + 1) ? Lp[1] : 0.0;
  out[3] = in(x - 1) ? Lp[3] : 0.0;
  out[2] = Lp[2];
  out[4] = Lp[4];
  out[5] = top ? r * Lp[5] + (in(xsp) ? omr * Lq[0] : 0.0) : (in(x + 1) ? Lp[5] : 0.0);
  out[6] = top ? r * Lp[6] + (in(xsm) ? omr * Lq[1] : 0.0) : (in(x - 1) ? Lp[6] : 0.0);
  out[7] = bot ? r * Lp[7] + (in(xsm) ? omr * Lq[2] : 0.0) : (in(x - 1) ? Lp[7] : 0.0);
  out[8] = bot ? r * Lp[8] + (in(xsp) ? omr * Lq[3] : 0.0) : (in(x + 1) ? Lp[8] : 0.0);
}

// Inputs of the reverse of one ghost row y (inlet or outlet): the adjoint of
// the three ghost directions that enter the channel, read from lp at the
// adjacent column c1 (with the specular corner terms of Eq. 20), and the
// populations of P at c1 and at the next column c2.
struct GhostIn {
  double l0, lup, ldn, ltop, lbot;
  double f1[9], f2[9];
};

template <bool INLET>
__device__ __forceinline__ void ghost_sources(const AdjArgs& a, const double* __restrict__ lp,
                                              const double* __restrict__ P, int y, GhostIn& gi) {
  const int nx = a.g.nx, t = a.g.ny - 1;
  const int c1 = INLET ? 0 : nx - 1, c2 = INLET ? 1 : nx - 2;
  constexpr int d0 = INLET ? 1 : 3, dup = INLET ? 5 : 6, ddn = INLET ? 8 : 7;
  gi.l0 = lp[a.g.index(d0, c1, y)];
  gi.lup = lp[a.g.index(dup, c1, y < t ? y + 1 : t)];
  gi.ldn = lp[a.g.index(ddn, c1, y > 0 ? y - 1 : 0)];
  gi.ltop = lp[a.g.index(INLET ? 8 : 7, c1, t)];
  gi.lbot = lp[a.g.index(INLET ? 5 : 6, c1, 0)];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    gi.f1[i] = P[a.g.index(i, c1, y)];
    gi.f2[i] = P[a.g.index(i, c2, y)];
  }
}

// l1 / l2: the adjoint pushed back onto columns c1 / c2 at row y.
template <bool INLET>
__device__ __forceinline__ void ghost_apply(const AdjArgs& a, int y, const GhostIn& gi, double l1[9], double l2[9]) {
#pragma clang fp contract(off)
  const int t = a.g.ny - 1;
  const double omr = 1.0 - a.r;
  double lg[3];   // directions (1, 5, 8) at the inlet, (3, 6, 7) at the outlet
  lg[0] = gi.l0;
  lg[1] = y + 1 <= t ? gi.lup : ((y == t && a.shift) ? omr * gi.ltop : 0.0);
  lg[2] = y - 1 >= 0 ? gi.ldn : ((y == 0 && a.shift) ? omr * gi.lbot : 0.0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    l1[i] = 0.0;
    l2[i] = 0.0;
  }
  ghost_vjp<INLET>(gi.f1, gi.f2, INLET ? a.rho_in : a.rho_out, lg, l1, l2);
}

// Adds the ghost-row reverse to out[9] for nodes in the first two / last two
// columns (XB = 1 only).
__device__ __forceinline__ void ghost_add(const AdjArgs& a, int x, int y, bool need_in, bool need_out,
                                          const GhostIn& gi, const GhostIn& go, double out[9]) {
#pragma clang fp contract(off)
  const int nx = a.g.nx;
  if (need_in) {
    double l1[9], l2[9];
    ghost_apply<true>(a, y, gi, l1, l2);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] += (x == 0) ? l1[i] : l2[i];
  }
  if (need_out) {
    double l1[9], l2[9];
    ghost_apply<false>(a, y, go, l1, l2);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] += (x == nx - 1) ? l1[i] : l2[i];
  }
}

// The whole transposed gather of one node (any column).
__device__ __forceinline__ void transposed_gather(const AdjArgs& a, const double* __restrict__ lp,
                                                  const double* __restrict__ P, int x, int y, double out[9]) {
  const int nx = a.g.nx;
  const bool need_in = x <= 1, need_out = x >= nx - 2;
  GhostIn gi, go;
  if (need_in) ghost_sources<true>(a, lp, P, y, gi);
  if (need_out) ghost_sources<false>(a, lp, P, y, go);
  double Lp[9], Lq[4];
  tg_sources<1>(a, lp, x, y, Lp, Lq);
  tg_combine<1>(a, x, y, Lp, Lq, out);
  ghost_add(a, x, y, need_in, need_out, gi, go, out);
}

// ---------------------------------------------------------------------------
// One reverse step n.  lambda_{n+1}(x, y) is either pulled on the fly from
// lpre_{n+1} (PULL: the transposed gather of step n + 1, ghosts at P_{n+1})
// or read from a.lam.  Then lpre_n = (dC/dpre_n)^T lambda_{n+1} at
// pre_n = G(P_n), the rate sensitivities of each column flow through
// s(tau(Kn(rho_c))) into lpre_n at the centre rows and into dL/da, dL/dA2,
// and wall rows add lpre . dpre/dr to dL/dr.  Up to ny = RY each thread owns
// one node and keeps it in registers across the column reductions.
// ---------------------------------------------------------------------------
// Workgroup scratch of the reverse step: centre-row densities, per-row rate
// sensitivities and per-column results.
template <int RY>
struct AdjShared {
  static constexpr int CX = 256 / RY;
  double rcr[2][CX];
  double nu[RY][CX], q[RY][CX], rr[RY][CX];
  double lrc[CX], ca[CX], cA2[CX], cr[CX];
};

// Gathered state and pulled adjoint of node (x, y): all loads first, then
// the arithmetic.  XB = 3 for interior workgroups (columns 2 .. nx - 3, no
// boundary code), XB = 1 for the others.
template <int XB, bool PULL>
__device__ __forceinline__ void adj_node_inputs(const AdjArgs& a, const Gather<XB == 3 ? 3 : 2, View>& gat, int x,
                                                int y, double f[9], double lo[9], double A[9], double B[4]) {
#pragma clang fp contract(off)
  const int nx = a.g.nx;
  const bool need_in = XB == 1 && PULL && x <= 1;
  const bool need_out = XB == 1 && PULL && x >= nx - 2;
  GhostIn gi, go;
  if (need_in) ghost_sources<true>(a, a.lin, a.Pn1, y, gi);
  if (need_out) ghost_sources<false>(a, a.lin, a.Pn1, y, go);
  double Lp[9], Lq[4];
  gat.template load_sources<false>(x, y, A, B);
  if (PULL) {
    tg_sources<XB>(a, a.lin, x, y, Lp, Lq);
  } else {
    const size_t base = a.g.index(0, x, y);
    const size_t stride = (size_t)1 << a.g.lshift;
#pragma unroll
    for (int i = 0; i < 9; ++i) lo[i] = a.lam[base + i * stride];
  }
  gat.combine(y, A, B, f);
  if (PULL) {
    tg_combine<XB>(a, x, y, Lp, Lq, lo);
    if (XB == 1) ghost_add(a, x, y, need_in, need_out, gi, go, lo);
  }
}

template <int RY, bool PULL, int XB>
__device__ __forceinline__ void adj_columns(const AdjArgs& a, const Gather<XB == 3 ? 3 : 2, View>& gat, int blk,
                                            AdjShared<RY>& sh) {
#pragma clang fp contract(off)
  constexpr int CX = 256 / RY;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int x = blk * CX + tx;
  const int nx = a.g.nx, ny = a.g.ny;
  const bool lead = tx == 0 && ty == 0;
  // this workgroup's running gradient partials, fetched early
  double gp0 = 0.0, gp1 = 0.0, gp2 = 0.0;
  if (lead) {
    gp0 = a.gpart[3 * blk];
    gp1 = a.gpart[3 * blk + 1];
    gp2 = a.gpart[3 * blk + 2];
  }
  const int yc = ny / 2;
  const bool even = (ny & 1) == 0;
  const size_t stride = (size_t)1 << a.g.lshift;
  const bool one = ny <= RY;   // one node per thread
  double f[9], lo[9], A[9], B[4];
  bool active = false;
  if (one) {
    active = x < nx && ty < ny;
    if (active) {
      adj_node_inputs<XB, PULL>(a, gat, x, ty, f, lo, A, B);
      if (ty == yc) sh.rcr[0][tx] = sum9(f);
      if (even && ty == yc - 1) sh.rcr[1][tx] = sum9(f);
    }
  } else if (ty < 2 && x < nx && (ty == 0 || even)) {
    double g[9];
    gat.flat(x, yc - ty, g);
    sh.rcr[ty][tx] = sum9(g);
  }
  __syncthreads();
  double snu = 0.0, sq = 0.0, kn = 0.0, tt = 0.0, rc = 1.0;
  if (x < nx) {
    rc = even ? 0.5 * (sh.rcr[1][tx] + sh.rcr[0][tx]) : sh.rcr[0][tx];
    local_rates(a.kn, a.rho_out, rc, a.c_tau, a.a, a.A2, a.tq_den, snu, sq, kn, tt);
  }
  // Derivatives of the column's rates, needed once its sums are in:
  //   s_nu = 1/(1/2 + tt),  s_q = 1/(1/2 + 3/(D tt) + 4 pi A2 tt / D)   (Eqs. 18, 21)
  //   tt = c_tau Kn / (1 + a Kn),  Kn = Kn_out rho_out / rho_c
  double k_nu_rc = 0.0, k_q_rc = 0.0, k_nu_a = 0.0, k_q_a = 0.0, k_q_A2 = 0.0;
  if (ty == 0 && x < nx) {
    const double D = a.tq_den;
    const double dsnu_dtt = -snu * snu;
    const double dsq_dtt = (-sq * sq) * (4.0 * M_PI * a.A2 / D - 3.0 / (D * tt * tt));
    const double den = 1.0 + a.a * kn;
    const double dtt_drc = a.c_tau / (den * den) * (-kn / rc);
    const double dtt_da = -a.c_tau * kn * kn / (den * den);
    k_nu_rc = dsnu_dtt * dtt_drc;
    k_q_rc = dsq_dtt * dtt_drc;
    k_nu_a = dsnu_dtt * dtt_da;
    k_q_a = dsq_dtt * dtt_da;
    k_q_A2 = (-sq * sq) * (4.0 * M_PI * tt / D);
  }
  const Rates s{a.s3, snu, sq, a.s8};
  double acc_nu = 0.0, acc_q = 0.0, acc_r = 0.0;
  double lf[9];
  bool hold = false;   // this thread's centre-row lpre waits for the rate correction
  if (one) {
    if (active) {
      double lsnu, lsq;
      collide_vjp(f, lo, s, lf, lsnu, lsq);
      acc_nu = lsnu;
      acc_q = lsq;
      acc_r = gat.wall_dr(ty, A, B, lf);
      hold = ty == yc || (even && ty == yc - 1);
      if (!hold) {
        const size_t base = a.g.index(0, x, ty);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.lpre[base + i * stride] = lf[i];
      }
    }
  } else if (x < nx) {
    for (int y = ty; y < ny; y += RY) {
      double g[9], l[9], lg[9], Ay[9], By[4];
      adj_node_inputs<XB, PULL>(a, gat, x, y, g, l, Ay, By);
      double lsnu, lsq;
      collide_vjp(g, l, s, lg, lsnu, lsq);
      acc_nu += lsnu;
      acc_q += lsq;
      acc_r += gat.wall_dr(y, Ay, By, lg);
      const size_t base = a.g.index(0, x, y);
#pragma unroll
      for (int i = 0; i < 9; ++i) a.lpre[base + i * stride] = lg[i];
    }
  }
  sh.nu[ty][tx] = acc_nu;
  sh.q[ty][tx] = acc_q;
  sh.rr[ty][tx] = acc_r;
  __syncthreads();
  const double w = even ? 0.5 : 1.0;
  if (ty == 0) {
    double da = 0.0, dA2 = 0.0, dr = 0.0, l_rc = 0.0;
    if (x < nx) {
      double lnu = sh.nu[0][tx], lq = sh.q[0][tx];
      dr = sh.rr[0][tx];
      for (int k = 1; k < RY; ++k) {
        lnu += sh.nu[k][tx];
        lq += sh.q[k][tx];
        dr += sh.rr[k][tx];
      }
      l_rc = k_nu_rc * lnu + k_q_rc * lq;
      da = k_nu_a * lnu + k_q_a * lq;
      dA2 = k_q_A2 * lq;
      // rho_c = mean of the centre rows of pre: l_rc reaches every population
      // there; centre rows that are wall rows also carry an r dependence.
      double lp[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) lp[i] = w * l_rc;
      for (int k = 0; k < (even ? 2 : 1); ++k) {
        const int yy = yc - k;
        if (yy == 0 || yy == ny - 1) dr += wall_dr(gat, x, yy, lp);
        if (!one) {
          const size_t base = a.g.index(0, x, yy);
#pragma unroll
          for (int i = 0; i < 9; ++i) a.lpre[base + i * stride] += lp[i];
        }
      }
    }
    sh.lrc[tx] = l_rc;
    sh.ca[tx] = da;
    sh.cA2[tx] = dA2;
    sh.cr[tx] = dr;
  }
  __syncthreads();
  if (hold) {
    const double add = w * sh.lrc[tx];
    const size_t base = a.g.index(0, x, ty);
#pragma unroll
    for (int i = 0; i < 9; ++i) a.lpre[base + i * stride] = lf[i] + add;
  }
  if (lead) {
    double sa = 0.0, sA2 = 0.0, sr = 0.0;
    for (int k = 0; k < CX; ++k) {
      sa += sh.ca[k];
      sA2 += sh.cA2[k];
      sr += sh.cr[k];
    }
    a.gpart[3 * blk] = gp0 + sa;
    a.gpart[3 * blk + 1] = gp1 + sA2;
    a.gpart[3 * blk + 2] = gp2 + sr;
  }
}

// The reverse step, dispatched per workgroup: workgroups whose columns all
// lie in 2 .. nx - 3 run with no x-boundary code; the others read the ghost
// columns of P_n from a.gh and reverse the ghost rows of P_{n+1} in place.
template <int RY, bool PULL>
__global__ __launch_bounds__(256) void k_adj_step(AdjArgs a) {
  constexpr int CX = 256 / RY;
  __shared__ AdjShared<RY> sh;
  const View v{a.P, a.g};
  const double omr = 1.0 - a.r;
  const int ny = a.g.ny;
  const int blk = logical_block(a.xcd_remap);
  const bool interior = blk > 0 && (blk + 1) * CX <= a.g.nx - 2;
  if (interior)
    adj_columns<RY, PULL, 3>(a, Gather<3, View>{v, a.r, omr, a.shift, a.rho_in, a.rho_out}, blk, sh);
  else
    adj_columns<RY, PULL, 1>(a, Gather<2, View>{v, a.r, omr, a.shift, a.rho_in, a.rho_out, a.gh, a.gh + 9 * ny},
                             blk, sh);
}

// lambda_n = G^T lpre (+ reverse of the ghost columns), one thread per node.
__global__ __launch_bounds__(256) void k_adj_gather(AdjArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= a.g.nx) return;
  double out[9];
  transposed_gather(a, a.lpre, a.P, x, y, out);
#pragma unroll
  for (int i = 0; i < 9; ++i) a.out[a.g.index(i, x, y)] = out[i];
}

// Ghost columns of nstate states into gh[k][2][9][ny]: state 0 at `first`,
// state k >= 1 at rest + (k - 1) * S.  One workgroup per state.
__global__ __launch_bounds__(256) void k_ghosts(const double* __restrict__ first, const double* __restrict__ rest,
                                                size_t S, Geo g, double rho_in, double rho_out,
                                                double* __restrict__ gh) {
  const int k = blockIdx.x;
  const View v{k == 0 ? first : rest + (size_t)(k - 1) * S, g};
  const int ny = g.ny;
  double* out = gh + (size_t)k * 18 * ny;
  for (int j = threadIdx.x; j < 2 * ny; j += blockDim.x) {
    const bool inlet = j < ny;
    const int y = inlet ? j : j - ny;
    double gr[9];
    ghost_row(v, inlet, y, inlet ? rho_in : rho_out, gr);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[(inlet ? 0 : 9 * ny) + i * ny + y] = gr[i];
  }
}

// Loss of the final state from per-column sums m(x) and rho_c(x):
// diff(x) = dp(x) - dp*(x); scal[0] = L, scal[1] = m - m*, scal[2] = m.
__global__ __launch_bounds__(256) void k_adj_loss(const double* __restrict__ m, const double* __restrict__ rhoc,
                                                  const double* __restrict__ dpt, int nx, double rho_in,
                                                  double rho_out, double m_target, double* __restrict__ diff,
                                                  double* __restrict__ scal) {
#pragma clang fp contract(off)
  __shared__ double s[256];
  const double p_out = rho_out / 3.0, p_in = rho_in / 3.0;
  double acc = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) {
    const double pl = p_in - (p_in - p_out) * ((double)x + 0.5) / (double)nx;
    const double dp = (rhoc[x] / 3.0 - pl) / p_out;
    const double d = dp - dpt[x];
    diff[x] = d;
    acc += d * d;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mo = m[nx - 1];
    const double dm = mo - m_target;
    const double q = dm / m_target;
    scal[0] = s[0] / (double)nx + q * q;
    scal[1] = dm;
    scal[2] = mo;
  }
}

// dL/dpre of the final state: centre rows from the dp term, outlet column
// from the mass-flow term (m = sum_y sum_i e_ix pre_i there, F = 0).  The
// final gather itself depends on r at the wall rows: each wall node writes
// its lpre . dpre/dr to dr_wall[y == 0 ? x : nx + x].
__global__ void k_adj_seed(AdjArgs a, const double* __restrict__ diff, const double* __restrict__ scal,
                           double m_target, double* __restrict__ dr_wall) {
#pragma clang fp contract(off)
  const Geo g = a.g;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const int ny = g.ny, yc = ny / 2;
  const bool even = (ny & 1) == 0;
  const double p_out = a.rho_out / 3.0;
  double c = 0.0;
  if (y == yc || (even && y == yc - 1))
    c = (even ? 0.5 : 1.0) * (2.0 / (double)g.nx) * diff[x] / (3.0 * p_out);
  const double cm = (x == g.nx - 1) ? 2.0 * scal[1] / (m_target * m_target) : 0.0;
  double lp[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    lp[i] = c + cm * (double)ex_of(i);
    a.lpre[g.index(i, x, y)] = lp[i];
  }
  if (y == 0 || y == ny - 1) {
    const Gather<1, View> gat{{a.P, g}, a.r, 1.0 - a.r, a.shift, a.rho_in, a.rho_out};
    dr_wall[(y == 0 ? 0 : g.nx) + x] = wall_dr(gat, x, y, lp);
  }
}

// Add the fixed-order sum of the final-gather r terms to the first partial.
__global__ __launch_bounds__(256) void k_adj_seed_dr(const double* __restrict__ dr_wall, int n,
                                                     double* __restrict__ gpart) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += dr_wall[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gpart[2] += s[0];
}

__global__ void k_fill(double* p, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Sum the per-block gradient partials in a fixed order.
__global__ __launch_bounds__(64) void k_adj_grad_sum(const double* __restrict__ gpart, int nblk, double* __restrict__ out) {
  if (threadIdx.x < 3) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += gpart[3 * b + threadIdx.x];
    out[threadIdx.x] = acc;
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

#define ADJ_HIP(call)                                                      \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      char m_[256];                                                        \
      snprintf(m_, sizeof(m_), "%s: %s", #call, hipGetErrorString(e_));    \
      return clb::set_error(CLB_EHIP, m_);                                 \
    }                                                                      \
  } while (0)

}  // namespace
}  // namespace clb

struct clb_adjoint {
  clb_params p;
  clb_derived d;
  clb::Geo g;
  int32_t T, K, nck;
  size_t S;                // doubles per state buffer
  double* ck;              // [nck][S] checkpoints: P at steps 0, K, 2K, ...
  double* seg;             // [max(K, 2)][S] recompute / forward work buffers
  double* pT;              // P at step T
  double* lam[2];
  double* lpre;
  double* gh;              // [2][K][2][9][ny] ghost columns of the recomputed states
  double* gpart;           // [nblk][3]
  double* step_rates;      // [2][nx] row-kernel scratch of the forward steps
  double* step_ghosts;     // [2][9][ny] row-kernel scratch of the forward steps
  int cus;                 // compute units of the device (launch shapes)
  double* col;             // [6][nx]: m, su, rho_c, diff, final-gather r terms (2 nx)
  double* dpt;             // [nx] target dp*
  double* scal;            // [16]: loss, m - m*, m, grads
  int nblk;
  hipStream_t stream;      // caller's stream: forward run and reverse sweep
  hipStream_t rstream;     // private stream: checkpoint recompute of the next segment
  hipEvent_t ev_start, ev_ready[2], ev_free[2];
  double m_target;
  int forward_done;
  double host_scal[8];
};

namespace {

struct AdjLayout {
  size_t S, total, gh;
  int nck, nseg, nblk;
};

AdjLayout adj_layout(const clb_params* p, int32_t T, int32_t K) {
  AdjLayout L{};
  const clb::Geo g = clb::make_geo(p->nx, p->ny);
  L.S = g.size();
  L.nck = (T + K - 1) / K;
  // two sets of K - 1 recompute buffers (segment s recomputes while s + 1 reverses)
  L.nseg = 2 * (K - 1) < 2 ? 2 : 2 * (K - 1);
  const int cx = 256 / clb::adj_rows(p->ny);
  L.nblk = (p->nx + cx - 1) / cx;
  const size_t buf = clb::align256(L.S * sizeof(double));
  const size_t col = clb::align256((size_t)p->nx * sizeof(double));
  L.gh = clb::align256(2 * (size_t)K * 18 * (size_t)p->ny * sizeof(double));
  // + forward-step scratch of the row kernel: two per-column arrays and [2][9][ny]
  L.total = ((size_t)L.nck + (size_t)L.nseg + 4) * buf + L.gh + 7 * col +
            clb::align256((size_t)L.nblk * 3 * sizeof(double)) + clb::align256(16 * sizeof(double)) +
            2 * col + clb::align256(18 * (size_t)p->ny * sizeof(double));
  return L;
}

clb::StepArgs adj_step_args(const clb_adjoint* a, const double* src, double* dst) {
  clb::StepArgs s{};
  s.src = src;
  s.dst = dst;
  s.g = a->g;
  s.mode = 1;
  s.shift = a->p.cbbsr_shift;
  s.xcd_remap = 1;
  s.r = a->d.r;
  s.s3 = a->p.s3;
  s.snu = a->d.s_nu;
  s.sq = a->d.s_q;
  s.s8 = a->p.s8;
  s.kn = a->p.kn;
  s.a = a->p.a;
  s.A2 = a->p.A2;
  s.tq_den = a->p.tq_den;
  s.c_tau = std::sqrt(6.0 / M_PI) * (double)a->p.ny;
  s.rho_in = a->p.p_ratio * a->p.rho_out;
  s.rho_out = a->p.rho_out;
  // large grids take the row kernel; forward steps and the recompute never
  // run at the same time, so they share this scratch
  s.col_rates = a->step_rates;
  s.ghosts = a->step_ghosts;
  s.cus = a->cus;
  return s;
}

clb::AdjArgs adj_args(const clb_adjoint* a, const double* P, double* lpre) {
  clb::AdjArgs r{};
  r.P = P;
  r.lpre = lpre;
  r.gpart = a->gpart;
  r.g = a->g;
  r.shift = a->p.cbbsr_shift;
  r.r = a->d.r;
  r.s3 = a->p.s3;
  r.s8 = a->p.s8;
  r.kn = a->p.kn;
  r.a = a->p.a;
  r.A2 = a->p.A2;
  r.tq_den = a->p.tq_den;
  r.c_tau = std::sqrt(6.0 / M_PI) * (double)a->p.ny;
  r.rho_in = a->p.p_ratio * a->p.rho_out;
  r.rho_out = a->p.rho_out;
  r.xcd_remap = 1;
  return r;
}

clb_status step(clb_adjoint* a, const double* src, double* dst, hipStream_t st) {
  const clb::StepArgs s = adj_step_args(a, src, dst);
  ADJ_HIP(clb::launch_step(s, 256, st));
  return CLB_OK;
}

clb_status step(clb_adjoint* a, const double* src, double* dst) { return step(a, src, dst, a->stream); }

// State n of segment s when its recompute uses buffer set `set`.
double* seg_state(clb_adjoint* a, int s, int set, int n) {
  const int start = s * a->K;
  if (n == start) return a->ck + (size_t)s * a->S;
  return a->seg + ((size_t)set * (size_t)(a->K - 1) + (size_t)(n - start - 1)) * a->S;
}

// Ghost columns of state n of a segment recomputed into buffer set `set`.
double* seg_ghosts(clb_adjoint* a, int set, int k) {
  return a->gh + ((size_t)set * (size_t)a->K + (size_t)k) * 18 * (size_t)a->p.ny;
}

// Recompute the states of segment s from its checkpoint on the private
// stream, build their ghost columns, then mark buffer set `set` ready.
clb_status recompute(clb_adjoint* a, int s, int set) {
  const int start = s * a->K;
  const int end = (start + a->K < a->T) ? start + a->K : a->T;
  for (int n = start; n + 1 < end; ++n) {
    clb_status st = step(a, seg_state(a, s, set, n), seg_state(a, s, set, n + 1), a->rstream);
    if (st != CLB_OK) return st;
  }
  clb::k_ghosts<<<end - start, 256, 0, a->rstream>>>(seg_state(a, s, set, start),
                                                     a->seg + (size_t)set * (size_t)(a->K - 1) * a->S, a->S, a->g,
                                                     a->p.p_ratio * a->p.rho_out, a->p.rho_out, seg_ghosts(a, set, 0));
  ADJ_HIP(hipGetLastError());
  ADJ_HIP(hipEventRecord(a->ev_ready[set], a->rstream));
  return CLB_OK;
}

template <bool PULL>
clb_status launch_adj_step(clb_adjoint* a, const clb::AdjArgs& r) {
  const int ry = clb::adj_rows(a->p.ny), cx = 256 / ry;
  if (ry == 16)
    clb::k_adj_step<16, PULL><<<a->nblk, dim3(cx, ry), 0, a->stream>>>(r);
  else if (ry == 32)
    clb::k_adj_step<32, PULL><<<a->nblk, dim3(cx, ry), 0, a->stream>>>(r);
  else
    clb::k_adj_step<64, PULL><<<a->nblk, dim3(cx, ry), 0, a->stream>>>(r);
  ADJ_HIP(hipGetLastError());
  return CLB_OK;
}

// Reverse step n of the sweep: lpre_n from lpre_{n+1} (pulled, ghosts at
// P_{n+1}) and the state P_n with its ghost columns gh.
clb_status reverse_step(clb_adjoint* a, const double* Pn, const double* gh, const double* Pn1,
                        const double* lpre_next, double* lpre_out) {
  clb::AdjArgs r = adj_args(a, Pn, lpre_out);
  r.gh = gh;
  r.Pn1 = Pn1;
  r.lin = lpre_next;
  return launch_adj_step<true>(a, r);
}

// Observables and loss of the state P (pre-collision at its time level).
clb_status loss_of(clb_adjoint* a, const double* P) {
  clb::DiagArgs d{};
  d.src = P;
  d.g = a->g;
  d.mode = 1;
  d.shift = a->p.cbbsr_shift;
  d.r = a->d.r;
  d.rho_in = a->p.p_ratio * a->p.rho_out;
  d.rho_out = a->p.rho_out;
  const int nx = a->p.nx;
  d.m = a->col;
  d.su = a->col + nx;
  d.rhoc = a->col + 2 * nx;
  ADJ_HIP(clb::launch_column_sums(d, a->stream));
  clb::k_adj_loss<<<1, 256, 0, a->stream>>>(a->col, a->col + 2 * nx, a->dpt, nx, d.rho_in, d.rho_out, a->m_target,
                                            a->col + 3 * nx, a->scal);
  ADJ_HIP(hipGetLastError());
  return CLB_OK;
}

}  // namespace

extern "C" {

clb_status clb_adjoint_workspace_size(const clb_params* p, int32_t T, int32_t K, size_t* bytes) {
  if (!bytes) return clb::set_error(CLB_EINVAL, "bytes: NULL");
  clb_status st = clb::validate_params(p, nullptr);
  if (st != CLB_OK) return st;
  if (p->xbc != CLB_X_PRESSURE) return clb::set_error(CLB_EINVAL, "xbc: the adjoint covers the pressure-driven channel");
  if (T < 1) return clb::set_error(CLB_EINVAL, "T: must be >= 1");
  if (K < 1 || K > T) return clb::set_error(CLB_EINVAL, "K: must lie in [1, T]");
  *bytes = adj_layout(p, T, K).total;
  return CLB_OK;
}

clb_status clb_adjoint_init(const clb_params* p, int32_t T, int32_t K, void* d_workspace, size_t bytes,
                            void* hip_stream, clb_adjoint** out) {
  if (!out) return clb::set_error(CLB_EINVAL, "out: NULL");
  *out = nullptr;
  size_t need = 0;
  clb_status st = clb_adjoint_workspace_size(p, T, K, &need);
  if (st != CLB_OK) return st;
  if (!d_workspace) return clb::set_error(CLB_EINVAL, "d_workspace: NULL");
  if (bytes < need) return clb::set_error(CLB_ENOMEM, "workspace: smaller than clb_adjoint_workspace_size");
  if ((st = clb::check_device_ptr(d_workspace, need, "d_workspace")) != CLB_OK) return st;
  clb_adjoint* a = new (std::nothrow) clb_adjoint();
  if (!a) return clb::set_error(CLB_ENOMEM, "host context allocation failed");
  a->p = *p;
  clb::validate_params(p, &a->d);
  a->g = clb::make_geo(p->nx, p->ny);
  a->T = T;
  a->K = K;
  const AdjLayout L = adj_layout(p, T, K);
  a->nck = L.nck;
  a->S = L.S;
  a->nblk = L.nblk;
  const size_t buf = clb::align256(L.S * sizeof(double));
  const size_t col = clb::align256((size_t)p->nx * sizeof(double));
  char* q = static_cast<char*>(d_workspace);
  a->ck = reinterpret_cast<double*>(q);
  q += (size_t)L.nck * buf;
  a->seg = reinterpret_cast<double*>(q);
  q += (size_t)L.nseg * buf;
  a->pT = reinterpret_cast<double*>(q);
  q += buf;
  a->lam[0] = reinterpret_cast<double*>(q);
  q += buf;
  a->lam[1] = reinterpret_cast<double*>(q);
  q += buf;
  a->lpre = reinterpret_cast<double*>(q);
  q += buf;
  a->gh = reinterpret_cast<double*>(q);
  q += L.gh;
  a->col = reinterpret_cast<double*>(q);
  q += 6 * col;   // m, su, rho_c, diff, final-gather r terms (2 nx)
  a->dpt = reinterpret_cast<double*>(q);
  q += col;
  a->gpart = reinterpret_cast<double*>(q);
  q += clb::align256((size_t)L.nblk * 3 * sizeof(double));
  a->scal = reinterpret_cast<double*>(q);
  q += clb::align256(16 * sizeof(double));
  a->step_rates = reinterpret_cast<double*>(q);
  a->step_ghosts = reinterpret_cast<double*>(q + 2 * col);
  a->stream = static_cast<hipStream_t>(hip_stream);
  a->forward_done = 0;
  a->cus = clb::device_cus();
  hipError_t e = hipStreamCreateWithFlags(&a->rstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&a->ev_start, hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&a->ev_ready[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a->ev_free[k], hipEventDisableTiming);
  }
  // Padding lanes of every buffer are never read, but start them at zero.
  if (e == hipSuccess) {
    clb::k_fill<<<1024, 256, 0, a->stream>>>(reinterpret_cast<double*>(d_workspace), need / sizeof(double), 0.0);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    clb_adjoint_destroy(a);
    return clb::set_error(CLB_EHIP, hipGetErrorString(e));
  }
  *out = a;
  return CLB_OK;
}

clb_status clb_adjoint_forward(clb_adjoint* a, const double* d_dp_target, double m_target, double* h_loss) {
  const clb::TraceRange trace("clb_adjoint_forward");
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  clb_status st = clb::check_device_ptr(d_dp_target, (size_t)a->p.nx * sizeof(double), "d_dp_target");
  if (st != CLB_OK) return st;
  if (!(std::isfinite(m_target) && m_target != 0.0)) return clb::set_error(CLB_EINVAL, "m_target: must be finite and != 0");
  a->m_target = m_target;
  ADJ_HIP(hipMemcpyAsync(a->dpt, d_dp_target, (size_t)a->p.nx * sizeof(double), hipMemcpyDeviceToDevice, a->stream));
  clb::InitArgs ia{};
  ia.dst = a->ck;
  ia.g = a->g;
  ia.kind = a->p.init;
  ia.rho0 = a->p.rho0;
  ia.ux0 = a->p.ux0;
  ia.uy0 = a->p.uy0;
  ia.rho_in = a->p.p_ratio * a->p.rho_out;
  ia.rho_out = a->p.rho_out;
  ia.amp = a->p.init_amp;
  ia.seed = a->p.seed;
  ADJ_HIP(clb::launch_init(ia, a->stream));
  double* w0 = a->seg;
  double* w1 = a->seg + a->S;
  const double* src = a->ck;
  for (int n = 0; n < a->T; ++n) {
    double* dst;
    if ((n + 1) == a->T)
      dst = a->pT;
    else if ((n + 1) % a->K == 0)
      dst = a->ck + (size_t)((n + 1) / a->K) * a->S;
    else
      dst = (src == w0) ? w1 : w0;
    if ((st = step(a, src, dst)) != CLB_OK) return st;
    src = dst;
  }
  if ((st = loss_of(a, a->pT)) != CLB_OK) return st;
  a->forward_done = 1;
  if (h_loss) {
    ADJ_HIP(hipMemcpyAsync(a->host_scal, a->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
    ADJ_HIP(hipStreamSynchronize(a->stream));
    *h_loss = a->host_scal[0];
  }
  return CLB_OK;
}

clb_status clb_adjoint_backward(clb_adjoint* a, double* h_grad) {
  const clb::TraceRange trace("clb_adjoint_backward");
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  if (!h_grad) return clb::set_error(CLB_EINVAL, "h_grad: NULL");
  if (!a->forward_done) return clb::set_error(CLB_ESTATE, "clb_adjoint_backward: run clb_adjoint_forward first");
  clb_status st;
  clb::k_fill<<<1, 256, 0, a->stream>>>(a->gpart, (size_t)a->nblk * 3, 0.0);
  // lambda_T = G^T dL/dpre_T
  const dim3 grid((unsigned)((a->g.nx + 255) / 256), (unsigned)a->g.ny);
  // lpre of the final gather (the loss seed); lpre buffers alternate between
  // a->lpre and a->lam[0] through the sweep.
  double* lbuf[2] = {a->lpre, a->lam[0]};
  {
    const clb::AdjArgs r = adj_args(a, a->pT, lbuf[0]);
    double* dr_wall = a->col + 4 * a->p.nx;   // 2 * nx entries (bottom, top)
    clb::k_fill<<<1, 256, 0, a->stream>>>(dr_wall, 2 * (size_t)a->p.nx, 0.0);
    clb::k_adj_seed<<<grid, 256, 0, a->stream>>>(r, a->col + 3 * a->p.nx, a->scal, a->m_target, dr_wall);
    clb::k_adj_seed_dr<<<1, 256, 0, a->stream>>>(dr_wall, 2 * a->p.nx, a->gpart);
  }
  ADJ_HIP(hipGetLastError());
  // Segments are reversed from the last to the first.  The recompute of
  // segment s - 1 (private stream, buffer set (s - 1) & 1) overlaps the
  // reverse sweep of segment s (caller's stream, set s & 1); events order a
  // set's reuse after the sweep that read it.
  ADJ_HIP(hipEventRecord(a->ev_start, a->stream));
  ADJ_HIP(hipStreamWaitEvent(a->rstream, a->ev_start, 0));
  if ((st = recompute(a, a->nck - 1, (a->nck - 1) & 1)) != CLB_OK) return st;
  int cur = 0;   // lbuf[cur] holds lpre_{n+1}
  for (int s = a->nck - 1; s >= 0; --s) {
    const int set = s & 1;
    if (s >= 1) {
      if (s + 1 <= a->nck - 1) ADJ_HIP(hipStreamWaitEvent(a->rstream, a->ev_free[(s - 1) & 1], 0));
      if ((st = recompute(a, s - 1, (s - 1) & 1)) != CLB_OK) return st;
    }
    ADJ_HIP(hipStreamWaitEvent(a->stream, a->ev_ready[set], 0));
    const int start = s * a->K;
    const int end = (start + a->K < a->T) ? start + a->K : a->T;
    for (int n = end - 1; n >= start; --n) {
      const double* Pn1 = n + 1 < end ? seg_state(a, s, set, n + 1)
                                      : (end == a->T ? a->pT : a->ck + (size_t)(s + 1) * a->S);
      if ((st = reverse_step(a, seg_state(a, s, set, n), seg_ghosts(a, set, n - start), Pn1, lbuf[cur],
                             lbuf[cur ^ 1])) != CLB_OK)
        return st;
      cur ^= 1;
    }
    ADJ_HIP(hipEventRecord(a->ev_free[set], a->stream));
  }
  clb::k_adj_grad_sum<<<1, 64, 0, a->stream>>>(a->gpart, a->nblk, a->scal + 4);
  ADJ_HIP(hipGetLastError());
  ADJ_HIP(hipMemcpyAsync(a->host_scal, a->scal + 4, 3 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
  ADJ_HIP(hipStreamSynchronize(a->stream));
  const double dA = a->host_scal[0], dA2 = a->host_scal[1], dr = a->host_scal[2];
  h_grad[0] = dA;
  // r tied to A1 through Eq. (21) unless given explicitly: dr/dA1 = -sqrt(pi/6) r^2
  h_grad[1] = std::isnan(a->p.r) ? dr * (-std::sqrt(M_PI / 6.0) * a->d.r * a->d.r) : 0.0;
  h_grad[2] = dA2;
  h_grad[3] = dr;
  return CLB_OK;
}

clb_status clb_adjoint_observables(clb_adjoint* a, double* d_dp, double* h_m) {
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  if (!a->forward_done) return clb::set_error(CLB_ESTATE, "clb_adjoint_observables: run clb_adjoint_forward first");
  const int nx = a->p.nx;
  if (d_dp) {
    clb_status st = clb::check_device_ptr(d_dp, (size_t)nx * sizeof(double), "d_dp");
    if (st != CLB_OK) return st;
    ADJ_HIP(clb::launch_pressure_dev(a->col + 2 * nx, nx, a->p.p_ratio * a->p.rho_out, a->p.rho_out, d_dp,
                                     a->stream));
  }
  if (h_m) {
    ADJ_HIP(hipMemcpyAsync(a->host_scal, a->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
    ADJ_HIP(hipStreamSynchronize(a->stream));
    *h_m = a->host_scal[2];
  }
  return CLB_OK;
}

clb_status clb_adjoint_final_state(clb_adjoint* a, double* d_out) {
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  if (!a->forward_done) return clb::set_error(CLB_ESTATE, "clb_adjoint_final_state: run clb_adjoint_forward first");
  clb_status st = clb::check_device_ptr(d_out, 9 * (size_t)a->p.nx * a->p.ny * sizeof(double), "d_out");
  if (st != CLB_OK) return st;
  ADJ_HIP(clb::launch_export(a->pT, a->g, d_out, a->stream));
  return CLB_OK;
}

clb_status clb_adjoint_vjp_step(clb_adjoint* a, const double* d_P, const double* d_lam_next, double* d_lam_prev,
                                double* h_grad3) {
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  const size_t bytes = 9 * (size_t)a->p.nx * a->p.ny * sizeof(double);
  clb_status st;
  if ((st = clb::check_device_ptr(d_P, bytes, "d_P")) != CLB_OK) return st;
  if ((st = clb::check_device_ptr(d_lam_next, bytes, "d_lam_next")) != CLB_OK) return st;
  if ((st = clb::check_device_ptr(d_lam_prev, bytes, "d_lam_prev")) != CLB_OK) return st;
  // Stage the inputs in the device layout (uses the recompute buffers).
  double* P = a->seg;
  double* lam = a->seg + a->S;
  ADJ_HIP(clb::launch_import(d_P, a->g, P, a->stream));
  ADJ_HIP(clb::launch_import(d_lam_next, a->g, lam, a->stream));
  clb::k_fill<<<1, 256, 0, a->stream>>>(a->gpart, (size_t)a->nblk * 3, 0.0);
  clb::k_ghosts<<<1, 256, 0, a->stream>>>(P, P, a->S, a->g, a->p.p_ratio * a->p.rho_out, a->p.rho_out, a->gh);
  {
    clb::AdjArgs r = adj_args(a, P, a->lpre);
    r.gh = a->gh;
    r.lam = lam;
    if ((st = launch_adj_step<false>(a, r)) != CLB_OK) return st;
    r.out = a->lam[1];
    const dim3 grid((unsigned)((a->g.nx + 255) / 256), (unsigned)a->g.ny);
    clb::k_adj_gather<<<grid, 256, 0, a->stream>>>(r);
    ADJ_HIP(hipGetLastError());
  }
  ADJ_HIP(clb::launch_export(a->lam[1], a->g, d_lam_prev, a->stream));
  clb::k_adj_grad_sum<<<1, 64, 0, a->stream>>>(a->gpart, a->nblk, a->scal + 4);
  ADJ_HIP(hipGetLastError());
  if (h_grad3) {
    ADJ_HIP(hipMemcpyAsync(a->host_scal, a->scal + 4, 3 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
    ADJ_HIP(hipStreamSynchronize(a->stream));
    h_grad3[0] = a->host_scal[0];
    h_grad3[1] = a->host_scal[1];
    h_grad3[2] = a->host_scal[2];
  }
  return CLB_OK;
}

clb_status clb_adjoint_destroy(clb_adjoint* a) {
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  (void)hipStreamSynchronize(a->stream);
  if (a->rstream) (void)hipStreamSynchronize(a->rstream);
  for (int k = 0; k < 2; ++k) {
    if (a->ev_ready[k]) (void)hipEventDestroy(a->ev_ready[k]);
    if (a->ev_free[k]) (void)hipEventDestroy(a->ev_free[k]);
  }
  if (a->ev_start) (void)hipEventDestroy(a->ev_start);
  if (a->rstream) (void)hipStreamDestroy(a->rstream);
  delete a;
  return CLB_OK;
}

}  // extern "C"
