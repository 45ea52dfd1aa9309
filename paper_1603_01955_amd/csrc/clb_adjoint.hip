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
//   k_adj_collide: recompute pre = G(P); lpre = (dC/dpre)^T lambda' per
//     node; per column, the rate sensitivities flow through
//     s(tau(Kn(rho_c))) back into lpre at the centre rows and into dL/da,
//     dL/dA2; wall rows add lpre . dpre/dr to dL/dr.
//   k_adj_gather: lambda = G^T lpre as a pull over the uses of each P_i(x, y)
//     (regular streaming, the CBBSR mixes, the reverse of the ghost
//     extrapolation at the first two and last two columns).
// The forward run keeps ceil(T/K) checkpoints; the backward sweep recomputes
// each segment of K steps from its checkpoint and then reverses it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <new>

#include "clb.h"
#include "clb_adjoint_device.hpp"
#include "clb_device.hpp"
#include "clb_gather.hpp"
#include "clb_internal.hpp"

namespace clb {
namespace {

constexpr int AX = 64;   // columns per block
constexpr int AY = 4;    // row lanes per block

struct AdjArgs {
  const double* P;       // state P_n (device layout)
  const double* lam;     // lambda_{n+1} (device layout)
  double* lpre;          // lpre (device layout)
  double* out;           // lambda_n (device layout)
  double* gpart;         // [blocks][3] accumulated (da, dA2, dr)
  Geo g;
  int shift;
  double r;
  double s3, s8;
  double kn, a, A2, tq_den, c_tau;
  double rho_in, rho_out;
};

__device__ __forceinline__ double sum9(const double f[9]) {
  return f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
}

// lpre . d pre / d r for the wall-replaced entries of node (x, y) (Eq. 20).
__device__ double wall_dr(const Gather<1, View>& gat, int x, int y, const double lp[9]) {
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

// Reverse of the collision and of the local-Kn rates for one step.
__global__ __launch_bounds__(AX * AY) void k_adj_collide(AdjArgs a) {
#pragma clang fp contract(off)
  __shared__ double s_nu[AX], s_q[AX], s_kn[AX], s_tt[AX], s_rc[AX];
  __shared__ double r_nu[AY][AX], r_q[AY][AX], r_r[AY][AX];
  __shared__ double c_a[AX], c_A2[AX], c_r[AX];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int x = blockIdx.x * AX + tx;
  const int ny = a.g.ny;
  const Gather<1, View> gat{{a.P, a.g}, a.r, 1.0 - a.r, a.shift, a.rho_in, a.rho_out};
  const int yc = ny / 2;
  const bool even = (ny & 1) == 0;
  if (ty == 0 && x < a.g.nx) {
    double f[9];
    gat(x, yc, f);
    double rc = sum9(f);
    if (even) {
      gat(x, yc - 1, f);
      rc = 0.5 * (sum9(f) + rc);
    }
    const double kn = a.kn * a.rho_out / rc;
    const double tt = a.c_tau * kn / (1.0 + a.a * kn);
    s_rc[tx] = rc;
    s_kn[tx] = kn;
    s_tt[tx] = tt;
    s_nu[tx] = 1.0 / (0.5 + tt);
    s_q[tx] = 1.0 / (0.5 + (3.0 + 4.0 * M_PI * tt * tt * a.A2) / (a.tq_den * tt));
  }
  __syncthreads();
  double acc_nu = 0.0, acc_q = 0.0, acc_r = 0.0;
  if (x < a.g.nx) {
    const Rates s{a.s3, s_nu[tx], s_q[tx], a.s8};
    for (int y = ty; y < ny; y += AY) {
      double f[9], lo[9], lf[9];
      gat(x, y, f);
      const size_t base = a.g.index(0, x, y);
      const size_t stride = (size_t)1 << a.g.lshift;
#pragma unroll
      for (int i = 0; i < 9; ++i) lo[i] = a.lam[base + i * stride];
      double lsnu, lsq;
      collide_vjp(f, lo, s, lf, lsnu, lsq);
      acc_nu += lsnu;
      acc_q += lsq;
      if (y == 0 || y == ny - 1) acc_r += wall_dr(gat, x, y, lf);
#pragma unroll
      for (int i = 0; i < 9; ++i) a.lpre[base + i * stride] = lf[i];
    }
  }
  r_nu[ty][tx] = acc_nu;
  r_q[ty][tx] = acc_q;
  r_r[ty][tx] = acc_r;
  __syncthreads();
  if (ty == 0) {
    double da = 0.0, dA2 = 0.0, dr = 0.0;
    if (x < a.g.nx) {
      double lnu = r_nu[0][tx], lq = r_q[0][tx];
      for (int k = 1; k < AY; ++k) {
        lnu += r_nu[k][tx];
        lq += r_q[k][tx];
      }
      // s_nu = 1/(1/2 + tt);  s_q = 1/(1/2 + 3/(D tt) + 4 pi A2 tt / D)   (Eqs. 18, 21)
      const double snu = s_nu[tx], sq = s_q[tx], tt = s_tt[tx], kn = s_kn[tx], rc = s_rc[tx];
      const double D = a.tq_den;
      const double l_tt = -snu * snu * lnu + (-sq * sq) * (4.0 * M_PI * a.A2 / D - 3.0 / (D * tt * tt)) * lq;
      const double den = 1.0 + a.a * kn;
      // tt = c_tau Kn / (1 + a Kn),  Kn = Kn_out rho_out / rho_c
      const double dtt_dkn = a.c_tau / (den * den);
      const double l_rc = l_tt * dtt_dkn * (-kn / rc);
      da = l_tt * (-a.c_tau * kn * kn / (den * den));
      dA2 = (-sq * sq) * (4.0 * M_PI * tt / D) * lq;
      // rho_c = mean of the (one or two) centre rows of pre: spread l_rc back.
      const double w = even ? 0.5 : 1.0;
      double lp[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) lp[i] = w * l_rc;
      const size_t stride = (size_t)1 << a.g.lshift;
      for (int k = 0; k < (even ? 2 : 1); ++k) {
        const int yy = yc - k;
        const size_t base = a.g.index(0, x, yy);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.lpre[base + i * stride] += lp[i];
        if (yy == 0 || yy == ny - 1) dr += wall_dr(gat, x, yy, lp);
      }
    }
    c_a[tx] = da;
    c_A2[tx] = dA2;
    c_r[tx] = dr;
  }
  __syncthreads();
  if (tx == 0 && ty == 0) {
    double sa = 0.0, sA2 = 0.0, sr = 0.0;
    for (int k = 0; k < AX; ++k) {
      sa += c_a[k];
      sA2 += c_A2[k];
      sr += c_r[k];
    }
    for (int j = 0; j < AY; ++j)
      for (int k = 0; k < AX; ++k) sr += r_r[j][k];
    double* gp = a.gpart + 3 * blockIdx.x;
    gp[0] += sa;
    gp[1] += sA2;
    gp[2] += sr;
  }
}

// lambda_n = G^T lpre (+ reverse of the ghost columns), one thread per node.
__global__ __launch_bounds__(256) void k_adj_gather(AdjArgs a) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int nx = a.g.nx, ny = a.g.ny, t = ny - 1;
  if (x >= nx) return;
  const double r = a.r, omr = 1.0 - a.r;
  auto L = [&](int i, int xx, int yy) { return a.lpre[a.g.index(i, xx, yy)]; };
  double out[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int ex = ex_of(i), ey = ey_of(i);
    double acc = 0.0;
    const int xd = x + ex, yd = y + ey;
    if (yd >= 0 && yd < ny) {
      if (xd >= 0 && xd < nx) acc += L(i, xd, yd);   // regular streaming use
    } else if (ey < 0) {                            // below the bottom wall (Eq. 20)
      if (i == 4) acc += L(2, x, 0);
      if (i == 7) {
        acc += r * L(5, x, 0);
        const int xs = a.shift ? x - 1 : x;            // pre6(xs) takes P7(xs + 1)
        if (xs >= 0) acc += omr * L(6, xs, 0);
      }
      if (i == 8) {
        acc += r * L(6, x, 0);
        const int xs = a.shift ? x + 1 : x;            // pre5(xs) takes P8(xs - 1)
        if (xs < nx) acc += omr * L(5, xs, 0);
      }
    } else {                                        // above the top wall (mirror)
      if (i == 2) acc += L(4, x, t);
      if (i == 5) {
        acc += r * L(7, x, t);
        const int xs = a.shift ? x + 1 : x;            // pre8(xs) takes P5(xs - 1)
        if (xs < nx) acc += omr * L(8, xs, t);
      }
      if (i == 6) {
        acc += r * L(8, x, t);
        const int xs = a.shift ? x - 1 : x;            // pre7(xs) takes P6(xs + 1)
        if (xs >= 0) acc += omr * L(7, xs, t);
      }
    }
    out[i] = acc;
  }
  // Reverse of the ghost columns: inlet ghost row y is built from columns 0, 1.
  if (x <= 1) {
    double lg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    lg[1] = L(1, 0, y);
    if (y + 1 <= t) lg[5] += L(5, 0, y + 1);
    if (y == t && a.shift) lg[5] += omr * L(8, 0, t);
    if (y - 1 >= 0) lg[8] += L(8, 0, y - 1);
    if (y == 0 && a.shift) lg[8] += omr * L(5, 0, 0);
    double f1[9], f2[9], l1[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, l2[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f1[i] = a.P[a.g.index(i, 0, y)];
      f2[i] = a.P[a.g.index(i, 1, y)];
    }
    ghost_vjp(f1, f2, a.rho_in, lg, l1, l2);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] += (x == 0) ? l1[i] : l2[i];
  }
  // Outlet ghost row y is built from columns nx - 1, nx - 2.
  if (x >= nx - 2) {
    const int c1 = nx - 1;
    double lg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    lg[3] = L(3, c1, y);
    if (y + 1 <= t) lg[6] += L(6, c1, y + 1);
    if (y == t && a.shift) lg[6] += omr * L(7, c1, t);
    if (y - 1 >= 0) lg[7] += L(7, c1, y - 1);
    if (y == 0 && a.shift) lg[7] += omr * L(6, c1, 0);
    double f1[9], f2[9], l1[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, l2[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f1[i] = a.P[a.g.index(i, c1, y)];
      f2[i] = a.P[a.g.index(i, nx - 2, y)];
    }
    ghost_vjp(f1, f2, a.rho_out, lg, l1, l2);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] += (x == c1) ? l1[i] : l2[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) a.out[a.g.index(i, x, y)] = out[i];
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
  double* gpart;           // [nblk][3]
  double* col;             // [6][nx]: m, su, rho_c, diff, final-gather r terms (2 nx)
  double* dpt;             // [nx] target dp*
  double* scal;            // [16]: loss, m - m*, m, grads
  int nblk;
  hipStream_t stream;
  double m_target;
  int forward_done;
  double host_scal[8];
};

namespace {

struct AdjLayout {
  size_t S, total;
  int nck, nseg, nblk;
};

AdjLayout adj_layout(const clb_params* p, int32_t T, int32_t K) {
  AdjLayout L{};
  const clb::Geo g = clb::make_geo(p->nx, p->ny);
  L.S = g.size();
  L.nck = (T + K - 1) / K;
  L.nseg = K < 2 ? 2 : K;
  L.nblk = (p->nx + clb::AX - 1) / clb::AX;
  const size_t buf = clb::align256(L.S * sizeof(double));
  const size_t col = clb::align256((size_t)p->nx * sizeof(double));
  L.total = ((size_t)L.nck + (size_t)L.nseg + 4) * buf + 7 * col + clb::align256((size_t)L.nblk * 3 * sizeof(double)) +
            clb::align256(16 * sizeof(double));
  return L;
}

clb::StepArgs adj_step_args(const clb_adjoint* a, const double* src, double* dst) {
  clb::StepArgs s{};
  s.src = src;
  s.dst = dst;
  s.g = a->g;
  s.mode = 1;
  s.shift = a->p.cbbsr_shift;
  s.xcd_remap = 0;
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
  return s;
}

clb::AdjArgs adj_args(const clb_adjoint* a, const double* P, const double* lam, double* out) {
  clb::AdjArgs r{};
  r.P = P;
  r.lam = lam;
  r.lpre = a->lpre;
  r.out = out;
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
  return r;
}

clb_status step(clb_adjoint* a, const double* src, double* dst) {
  const clb::StepArgs s = adj_step_args(a, src, dst);
  ADJ_HIP(clb::launch_step(s, 256, a->stream));
  return CLB_OK;
}

clb_status reverse_step(clb_adjoint* a, const double* P, const double* lam_next, double* lam_out) {
  const clb::AdjArgs r = adj_args(a, P, lam_next, lam_out);
  clb::k_adj_collide<<<a->nblk, dim3(clb::AX, clb::AY), 0, a->stream>>>(r);
  const dim3 grid((unsigned)((a->g.nx + 255) / 256), (unsigned)a->g.ny);
  clb::k_adj_gather<<<grid, 256, 0, a->stream>>>(r);
  ADJ_HIP(hipGetLastError());
  return CLB_OK;
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
  a->col = reinterpret_cast<double*>(q);
  q += 6 * col;   // m, su, rho_c, diff, final-gather r terms (2 nx)
  a->dpt = reinterpret_cast<double*>(q);
  q += col;
  a->gpart = reinterpret_cast<double*>(q);
  q += clb::align256((size_t)L.nblk * 3 * sizeof(double));
  a->scal = reinterpret_cast<double*>(q);
  a->stream = static_cast<hipStream_t>(hip_stream);
  a->forward_done = 0;
  // Padding lanes of every buffer are never read, but start them at zero.
  clb::k_fill<<<1024, 256, 0, a->stream>>>(reinterpret_cast<double*>(d_workspace), need / sizeof(double), 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete a;
    return clb::set_error(CLB_EHIP, hipGetErrorString(e));
  }
  *out = a;
  return CLB_OK;
}

clb_status clb_adjoint_forward(clb_adjoint* a, const double* d_dp_target, double m_target, double* h_loss) {
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
  if (!a) return clb::set_error(CLB_EINVAL, "adjoint: NULL");
  if (!h_grad) return clb::set_error(CLB_EINVAL, "h_grad: NULL");
  if (!a->forward_done) return clb::set_error(CLB_ESTATE, "clb_adjoint_backward: run clb_adjoint_forward first");
  clb_status st;
  clb::k_fill<<<1, 256, 0, a->stream>>>(a->gpart, (size_t)a->nblk * 3, 0.0);
  // lambda_T = G^T dL/dpre_T
  const dim3 grid((unsigned)((a->g.nx + 255) / 256), (unsigned)a->g.ny);
  {
    const clb::AdjArgs r = adj_args(a, a->pT, nullptr, a->lam[0]);
    double* dr_wall = a->col + 4 * a->p.nx;   // 2 * nx entries (bottom, top)
    clb::k_fill<<<1, 256, 0, a->stream>>>(dr_wall, 2 * (size_t)a->p.nx, 0.0);
    clb::k_adj_seed<<<grid, 256, 0, a->stream>>>(r, a->col + 3 * a->p.nx, a->scal, a->m_target, dr_wall);
    clb::k_adj_seed_dr<<<1, 256, 0, a->stream>>>(dr_wall, 2 * a->p.nx, a->gpart);
    clb::k_adj_gather<<<grid, 256, 0, a->stream>>>(r);
  }
  ADJ_HIP(hipGetLastError());
  int cur = 0;   // lam[cur] holds lambda_{n+1}
  for (int s = a->nck - 1; s >= 0; --s) {
    const int start = s * a->K;
    const int end = (start + a->K < a->T) ? start + a->K : a->T;
    auto buf = [&](int n) -> double* {
      return n == start ? a->ck + (size_t)s * a->S : a->seg + (size_t)(n - start - 1) * a->S;
    };
    for (int n = start; n + 1 < end; ++n)
      if ((st = step(a, buf(n), buf(n + 1))) != CLB_OK) return st;
    for (int n = end - 1; n >= start; --n) {
      if ((st = reverse_step(a, buf(n), a->lam[cur], a->lam[cur ^ 1])) != CLB_OK) return st;
      cur ^= 1;
    }
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
  if ((st = reverse_step(a, P, lam, a->lam[0])) != CLB_OK) return st;
  ADJ_HIP(clb::launch_export(a->lam[0], a->g, d_lam_prev, a->stream));
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
  delete a;
  return CLB_OK;
}

}  // extern "C"
