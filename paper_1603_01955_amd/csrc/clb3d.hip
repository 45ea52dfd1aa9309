// 3-D cascaded LB step for gas flow in a rectangular microduct (D3Q27, FP64),
// force-driven or pressure-driven, declared in include/clb3d.h.
//
// Method: the 2-D scheme of Liu & He (arXiv:1603.01955) carried to 3-D, the
// extension the paper names as future work (Section 4): pull streaming
// (Eq. 5) with the combined bounce-back / specular wall of Eq. (20) on the
// duct walls, then the cascaded collision (Eqs. 6-9, 13) in central-moment
// form.  Force-driven ducts (x periodic, Section 3.1): one kernel per step,
// gather, collide, store -- 216 B read and 216 B written per node update.
// Pressure-driven ducts (Section 3.2 carried to 3-D): per step the two ghost
// planes x = -1, x = nx (k3_ghosts), the relaxation rates of every
// cross-section from the local Knudsen number at its centre (k3_rates),
// then the step, which pulls across the inlet and outlet from the ghost
// planes.
//
// Device layout: each (y, z) row is cut into segments of L = min(1024, the
// next power of two >= nx) columns, and a segment stores its 27 directions
// one after the other, L values each: [nz][ny][segment][27][L].  A
// wavefront's loads of one direction are one contiguous 512-byte piece, and
// the 27 pieces of a row segment lie together (216 L bytes) instead of in 27
// planes far apart.  clb3_get_populations / clb3_set_populations convert
// from / to the ABI layout [27][nz][ny][nx].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "clb3d.h"
#include "clb_device.hpp"
#include "clb_internal.hpp"
#include "clb_trace.hpp"

namespace clb3 {
namespace {

struct Args {
  const double* src;    // post-collision populations at t - 1 (device layout)
  double* dst;          // post-collision populations at t
  int nx, ny, nz;
  int lshift, nseg;     // L = 2^lshift columns per row segment, nseg segments per row
  size_t plane;         // nx * ny * nz (logical nodes)
  int zwalls;           // 1: walls in z (duct), 0: z periodic (channel)
  int shift;            // Eq. (20) specular source displaced along the walls
  double r, omr;        // bounce-back fraction and 1 - r
  double gx, gy, gz;
  double sb, snu, sq, s8;
  // pressure-driven ducts (pressure = 1)
  int pressure;
  double rho_in, rho_out;   // boundary densities, p = rho / 3
  double kn, ab, A2, tq_den, c_tau;   // Kn_out, Eq. (18) a, B2, Eq. (21) denominator, sqrt(6/pi) ny
  double* ghosts;           // [2][nz][ny][27]: inlet plane x = -1, outlet plane x = nx
  double* col_rates;        // [2][nx]: s_nu(x), then s_q(x)
};

// Ghost population i of side (0 inlet, 1 outlet) at row y, layer z; the 27
// values of one row lie together.
__device__ __forceinline__ size_t ghost_row(const Args& a, int side, int y, int z) {
  return (((size_t)side * (size_t)a.nz + (size_t)z) * (size_t)a.ny + (size_t)y) * 27;
}

__device__ __forceinline__ double ghost(const Args& a, int side, int i, int y, int z) {
  return a.ghosts[ghost_row(a, side, y, z) + (size_t)i];
}

// Logical node number (the ABI order, x fastest).
__device__ __forceinline__ size_t node_index(const Args& a, int x, int y, int z) {
  return ((size_t)z * (size_t)a.ny + (size_t)y) * (size_t)a.nx + (size_t)x;
}

// Device-layout offset of direction 0 of node (x, y, z); direction i lies
// i << lshift further.
__device__ __forceinline__ size_t dev_index(const Args& a, int x, int y, int z) {
  const size_t seg = ((size_t)z * (size_t)a.ny + (size_t)y) * (size_t)a.nseg + (size_t)(x >> a.lshift);
  return ((seg * 27) << a.lshift) + (size_t)(x & ((1 << a.lshift) - 1));
}

// Pre-collision populations of node (x, y, z): pull streaming (Eq. 5), x
// periodic (PRESSURE false) or open at the inlet and outlet with the source
// taken from the ghost planes (PRESSURE true), z periodic or walled; where
// the source n - e lies behind the wall planes of a set S of axes, Eq. (20)
// carried to 3-D:
//   pre_e(n) = r P_{-e}(n) + (1 - r) P_{e'}(n - e_t),
// e' = e with its components along S reversed, e_t = e without them (the
// node itself when shift = 0); a displaced source beyond the inlet or the
// outlet is a ghost value.
// Pre-collision population of one direction (e, b, c), given at run time,
// at node (x, y, z), self = dev_index of the node: the rule of gather below
// for that direction alone (the rates kernel spreads the directions of a
// node over lanes).
template <bool PRESSURE>
__device__ __forceinline__ double pull(const Args& a, int x, int y, int z, size_t self, int e, int b, int c) {
#pragma clang fp contract(off)
  const double* __restrict__ P = a.src;
  const int i = (e + 1) + 3 * (b + 1) + 9 * (c + 1);
  int xs = x - e;
  if (!PRESSURE) xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
  const bool gh = PRESSURE && (xs < 0 || xs >= a.nx);   // the source lies on a ghost plane
  const int side = xs < 0 ? 0 : 1;
  const int ys = y - b;
  int zs = z - c;
  const bool oy = ys < 0 || ys >= a.ny;
  bool oz = false;
  if (a.zwalls)
    oz = zs < 0 || zs >= a.nz;
  else
    zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
  double v;
  if (!oy && !oz) {
    v = gh ? ghost(a, side, i, ys, zs) : P[((size_t)i << a.lshift) + dev_index(a, xs, ys, zs)];
  } else {
    const int i2 = (e + 1) + 3 * ((oy ? -b : b) + 1) + 9 * ((oz ? -c : c) + 1);
    const double bb = P[((size_t)(26 - i) << a.lshift) + self];
    const int sy = oy ? y : ys, sz = oz ? z : zs;
    double sp;
    if (gh && a.shift) {
      sp = ghost(a, side, i2, sy, sz);
    } else {
      const size_t sn = a.shift ? dev_index(a, xs, sy, sz) : self;
      sp = P[((size_t)i2 << a.lshift) + sn];
    }
    v = a.r * bb + a.omr * sp;
  }
  return v;
}

// The 27 pre-collision populations of node (x, y, z): pull for every
// direction, written out in full (the step's hot loop; the compiler keeps
// the wall and ghost tests of each direction apart).
template <bool PRESSURE>
__device__ __forceinline__ void gather(const Args& a, int x, int y, int z, double f[27]) {
#pragma clang fp contract(off)
  const double* __restrict__ P = a.src;
  const size_t self = dev_index(a, x, y, z);
#pragma unroll
  for (int c = -1; c <= 1; ++c) {
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
#pragma unroll
      for (int e = -1; e <= 1; ++e) {
        const int i = (e + 1) + 3 * (b + 1) + 9 * (c + 1);
        int xs = x - e;
        if (!PRESSURE) xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
        const bool gh = PRESSURE && (xs < 0 || xs >= a.nx);   // the source lies on a ghost plane
        const int side = xs < 0 ? 0 : 1;
        const int ys = y - b;
        int zs = z - c;
        const bool oy = ys < 0 || ys >= a.ny;
        bool oz = false;
        if (a.zwalls)
          oz = zs < 0 || zs >= a.nz;
        else
          zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
        if (!oy && !oz) {
          f[i] = gh ? ghost(a, side, i, ys, zs) : P[((size_t)i << a.lshift) + dev_index(a, xs, ys, zs)];
        } else {
          const int i2 = (e + 1) + 3 * ((oy ? -b : b) + 1) + 9 * ((oz ? -c : c) + 1);
          const double bb = P[((size_t)(26 - i) << a.lshift) + self];
          const int sy = oy ? y : ys, sz = oz ? z : zs;
          double sp;
          if (gh && a.shift) {
            sp = ghost(a, side, i2, sy, sz);
          } else {
            const size_t sn = a.shift ? dev_index(a, xs, sy, sz) : self;
            sp = P[((size_t)i2 << a.lshift) + sn];
          }
          f[i] = a.r * bb + a.omr * sp;
        }
      }
    }
  }
}

// gather for the mode of a (the diagnostics' kernels serve both).
__device__ __forceinline__ void gather_any(const Args& a, int x, int y, int z, double f[27]) {
  if (a.pressure)
    gather<true>(a, x, y, z, f);
  else
    gather<false>(a, x, y, z, f);
}

// Density and momentum of the populations (x, y, z components).
__device__ __forceinline__ void rho_j(const double f[27], double& rho, double& jx, double& jy, double& jz) {
#pragma clang fp contract(off)
  double s[9], t[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {   // row (b, c) along x
    s[k] = f[3 * k + 1] + (f[3 * k + 2] + f[3 * k]);
    t[k] = f[3 * k + 2] - f[3 * k];
  }
  rho = ((s[0] + s[1] + s[2]) + (s[3] + s[4] + s[5])) + (s[6] + s[7] + s[8]);
  jx = ((t[0] + t[1] + t[2]) + (t[3] + t[4] + t[5])) + (t[6] + t[7] + t[8]);
  jy = ((s[2] - s[0]) + (s[5] - s[3])) + (s[8] - s[6]);
  jz = ((s[6] - s[0]) + (s[7] - s[1])) + (s[8] - s[2]);
}

// The central-moment collision, in place on f[27] (slot A + 3B + 9C holds
// direction (A - 1, B - 1, C - 1), then moment order (A, B, C)).  Three
// passes of the one-axis transform of the 2-D step give the central moments
// k_pqr about u; relaxation (trace at s_b towards rho, deviator and shear at
// s_nu, third order at s_q, orders 4-6 at s8 towards rho c_p c_q c_r with
// c = (1, 0, 1/3), first order + rho F); three passes back.
template <bool FORCE>
__device__ __forceinline__ void collide(double f[27], const Args& a, double snu, double sq) {
#pragma clang fp contract(off)
  using clb::detail::axis_central;
  using clb::detail::axis_populations;
  double rho, jx, jy, jz;
  rho_j(f, rho, jx, jy, jz);
  const double inv = 1.0 / rho;
  const double ux = FORCE ? fma(jx, inv, 0.5 * a.gx) : jx * inv;
  const double uy = FORCE ? fma(jy, inv, 0.5 * a.gy) : jy * inv;
  const double uz = FORCE ? fma(jz, inv, 0.5 * a.gz) : jz * inv;
  const double ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const double tux = ux + ux, tuy = uy + uy, tuz = uz + uz;
  // forward: x, y, z
#pragma unroll
  for (int k = 0; k < 9; ++k)
    axis_central(f[3 * k], f[3 * k + 1], f[3 * k + 2], ux, ux2, tux, f[3 * k], f[3 * k + 1], f[3 * k + 2]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int o = p + 9 * c;
      axis_central(f[o], f[o + 3], f[o + 6], uy, uy2, tuy, f[o], f[o + 3], f[o + 6]);
    }
#pragma unroll
  for (int k = 0; k < 9; ++k) axis_central(f[k], f[k + 9], f[k + 18], uz, uz2, tuz, f[k], f[k + 9], f[k + 18]);

  // relaxation; k_pqr sits in slot p + 3 q + 9 r
  if (FORCE) {
    f[1] = f[1] + rho * a.gx;
    f[3] = f[3] + rho * a.gy;
    f[9] = f[9] + rho * a.gz;
  }
  const double third = 1.0 / 3.0;
  const double tr = (f[2] + f[6]) + f[18];
  const double tr1 = tr - a.sb * (tr - rho);
  const double onu = 1.0 - snu;
  const double mean = tr * third, mean1 = tr1 * third;
  f[2] = mean1 + onu * (f[2] - mean);
  f[6] = mean1 + onu * (f[6] - mean);
  f[18] = mean1 + onu * (f[18] - mean);
  f[4] = onu * f[4];     // k110
  f[10] = onu * f[10];   // k101
  f[12] = onu * f[12];   // k011
  const double oq = 1.0 - sq;
  // third order: k210 k120 k201 k021 k102 k012 k111
  f[5] = oq * f[5];
  f[7] = oq * f[7];
  f[11] = oq * f[11];
  f[15] = oq * f[15];
  f[19] = oq * f[19];
  f[21] = oq * f[21];
  f[13] = oq * f[13];
  // orders 4-6: k220 k202 k022 towards rho/9, k222 towards rho/27, the rest to 0
  const double e9 = rho * (1.0 / 9.0), e27 = rho * (1.0 / 27.0);
  f[8] = f[8] - a.s8 * (f[8] - e9);
  f[20] = f[20] - a.s8 * (f[20] - e9);
  f[24] = f[24] - a.s8 * (f[24] - e9);
  f[26] = f[26] - a.s8 * (f[26] - e27);
  const double o8 = 1.0 - a.s8;
  f[14] = o8 * f[14];    // k211
  f[16] = o8 * f[16];    // k121
  f[22] = o8 * f[22];    // k112
  f[17] = o8 * f[17];    // k221
  f[23] = o8 * f[23];    // k212
  f[25] = o8 * f[25];    // k122

  // back: z, y, x
#pragma unroll
  for (int k = 0; k < 9; ++k) axis_populations(f[k], f[k + 9], f[k + 18], uz, uz2, tuz, f[k], f[k + 9], f[k + 18]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int o = p + 9 * c;
      axis_populations(f[o], f[o + 3], f[o + 6], uy, uy2, tuy, f[o], f[o + 3], f[o + 6]);
    }
#pragma unroll
  for (int k = 0; k < 9; ++k)
    axis_populations(f[3 * k], f[3 * k + 1], f[3 * k + 2], ux, ux2, tux, f[3 * k], f[3 * k + 1], f[3 * k + 2]);
}

constexpr int kBX = 64, kBY = 4;

// Order of the step's workgroups.  The hardware deals consecutive
// workgroups to the eight XCDs in turn; logical block l = (b mod 8) per +
// b / 8 gives each XCD one contiguous range of l, which walks chunks of
// kChunkRows block rows (kChunkRows kBY rows of y): in a chunk z by z, in a
// plane block row by block row, in a block row x by x.  The x and y
// neighbours a workgroup pulls from then run on the same XCD at about the
// same time, and its z neighbours kChunkRows nbx workgroups before or after
// it, so the rows they share stay in that XCD's L2.
constexpr int kChunkRows = 8;

__device__ __forceinline__ void step_block(const Args& a, int& bx, int& by, int& z) {
  int l = (int)blockIdx.x;
  const int per = (int)gridDim.x >> 3;
  if (l < (per << 3)) l = (l & 7) * per + (l >> 3);
  const int nbx = (a.nx + kBX - 1) / kBX, nby = (a.ny + kBY - 1) / kBY;
  const int full = nby / kChunkRows;
  // workgroups of a full chunk; no more than the grid (below 2^31) holds
  const int per_chunk = a.nz * (nby < kChunkRows ? nby : kChunkRows) * nbx;
  int chunk = l / per_chunk, h = kChunkRows;
  int rem = l - chunk * per_chunk;
  if (chunk >= full) {   // the last, shorter chunk
    chunk = full;
    rem = l - full * per_chunk;
    h = nby - full * kChunkRows;
  }
  z = rem / (h * nbx);
  const int r2 = rem - z * (h * nbx);
  by = chunk * kChunkRows + r2 / nbx;
  bx = r2 - (r2 / nbx) * nbx;
}

template <bool FORCE, bool PRESSURE>
__global__ __launch_bounds__(kBX * kBY) void k3_step(Args a) {
  int bx, by, z;
  step_block(a, bx, by, z);
  const int x = bx * kBX + (threadIdx.x & (kBX - 1));
  const int y = by * kBY + (int)(threadIdx.x / kBX);
  if (x >= a.nx || y >= a.ny) return;
  double f[27];
  gather<PRESSURE>(a, x, y, z, f);
  if (PRESSURE)
    collide<FORCE>(f, a, a.col_rates[x], a.col_rates[a.nx + x]);
  else
    collide<FORCE>(f, a, a.snu, a.sq);
  const size_t n = dev_index(a, x, y, z);
#pragma unroll
  for (int i = 0; i < 27; ++i) __builtin_nontemporal_store(f[i], a.dst + ((size_t)i << a.lshift) + n);
}

// Macroscopic fields of the pre-collision state (Eqs. 12-13).
__global__ __launch_bounds__(kBX * kBY) void k3_moments(Args a, double* rho, double* ux, double* uy, double* uz) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * kBX + (threadIdx.x & (kBX - 1));
  const int y = blockIdx.y * kBY + (int)(threadIdx.x / kBX);
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  double f[27];
  gather_any(a, x, y, z, f);
  double r, jx, jy, jz;
  rho_j(f, r, jx, jy, jz);
  const size_t n = node_index(a, x, y, z);
  if (rho) rho[n] = r;
  if (ux) ux[n] = jx / r + 0.5 * a.gx;
  if (uy) uy[n] = jy / r + 0.5 * a.gy;
  if (uz) uz[n] = jz / r + 0.5 * a.gz;
}

// Per-workgroup partial sums of u_x (pre-collision state) over the nodes,
// in a fixed order: strided per-thread sums, wavefront butterflies, the four
// wavefront totals in order.
__global__ __launch_bounds__(256) void k3_ux_partial(Args a, double* partial) {
#pragma clang fp contract(off)
  __shared__ double s[4];
  double acc = 0.0;
  for (size_t n = blockIdx.x * (size_t)256 + threadIdx.x; n < a.plane; n += (size_t)gridDim.x * 256) {
    const int x = (int)(n % (size_t)a.nx);
    const size_t rest = n / (size_t)a.nx;
    const int y = (int)(rest % (size_t)a.ny);
    const int z = (int)(rest / (size_t)a.ny);
    double f[27];
    gather<false>(a, x, y, z, f);   // force-driven ducts only
    double r, jx, jy, jz;
    rho_j(f, r, jx, jy, jz);
    acc += jx / r + 0.5 * a.gx;
  }
  acc = clb::wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// One axis factor of the D3Q27 equilibrium f^eq_i(rho, u) = rho prod_axes
// w(e, u): w(0, u) = 2/3 - u^2, w(+-1, u) = (1/3 + u^2 +- u) / 2.  Along each
// axis the three factors have zeroth, first and second central moments 1, 0,
// 1/3, so the product has the equilibrium central moments rho c_p c_q c_r,
// c = (1, 0, 1/3), of the collision.
__device__ __forceinline__ double eq_axis(int e, double u) {
#pragma clang fp contract(off)
  return e == 0 ? 2.0 / 3.0 - u * u : 0.5 * ((1.0 / 3.0 + u * u) + (double)e * u);
}

// Sum over the 32 lanes of a half-wavefront, the same value (bitwise) in
// every lane: butterfly of fixed order.
__device__ __forceinline__ double group32_sum(double v) {
#pragma clang fp contract(off)
#pragma unroll
  for (int d = 16; d > 0; d >>= 1) v += __shfl_xor(v, d, 32);
  return v;
}

// Ghost planes of a pressure-driven duct, 32 lanes per (side, y, z), lane
// i < 27 for direction i: the inlet/outlet rule of Section 3.2 applied to
// every row of the cross-section,
//   ghost_i = f^eq_i(2 rho_b - rho_1, 2 u_1 - u_2) + P_i(c1) - f^eq_i(rho_1, u_1),
// rho_1, u_1 the density and velocity of the post-collision populations of
// the column next to the plane (c1 = 0 at the inlet, nx - 1 at the outlet),
// u_2 those of the column after it, rho_b = rho_in at the inlet, rho_out at
// the outlet.  The moments are lane sums over the group.
__global__ __launch_bounds__(256) void k3_ghosts(Args a) {
#pragma clang fp contract(off)
  const size_t cs = (size_t)a.ny * (size_t)a.nz;
  const int i = (int)(threadIdx.x & 31);
  const int ex = i % 3 - 1, ey = (i / 3) % 3 - 1, ez = i / 9 - 1;
  // whole 32-lane groups stay together through the loop and the shuffles
  for (size_t g = (blockIdx.x * (size_t)256 + threadIdx.x) >> 5; g < 2 * cs; g += (size_t)gridDim.x * 8) {
    const int side = g >= cs ? 1 : 0;
    const size_t yz = g - (side ? cs : 0);
    const int y = (int)(yz % (size_t)a.ny), z = (int)(yz / (size_t)a.ny);
    const int c1 = side ? a.nx - 1 : 0, c2 = side ? a.nx - 2 : 1;
    const double rho_b = side ? a.rho_out : a.rho_in;
    double f1 = 0.0, f2 = 0.0;
    if (i < 27) {
      f1 = a.src[((size_t)i << a.lshift) + dev_index(a, c1, y, z)];
      f2 = a.src[((size_t)i << a.lshift) + dev_index(a, c2, y, z)];
    }
    const double r1 = group32_sum(f1), r2 = group32_sum(f2);
    const double jx1 = group32_sum((double)ex * f1), jy1 = group32_sum((double)ey * f1),
                 jz1 = group32_sum((double)ez * f1);
    const double jx2 = group32_sum((double)ex * f2), jy2 = group32_sum((double)ey * f2),
                 jz2 = group32_sum((double)ez * f2);
    const double u1x = jx1 / r1, u1y = jy1 / r1, u1z = jz1 / r1;
    const double u2x = jx2 / r2, u2y = jy2 / r2, u2z = jz2 / r2;
    if (i < 27) {
      const double rg = 2.0 * rho_b - r1;
      const double eg = rg * eq_axis(ex, 2.0 * u1x - u2x) * eq_axis(ey, 2.0 * u1y - u2y) * eq_axis(ez, 2.0 * u1z - u2z);
      const double e1 = r1 * eq_axis(ex, u1x) * eq_axis(ey, u1y) * eq_axis(ez, u1z);
      a.ghosts[ghost_row(a, side, y, z) + (size_t)i] = eg + (f1 - e1);
    }
  }
}

// Pre-collision density at the centre of cross-section x: the mean over the
// middle row (odd ny) or the two middle rows (even ny) of the middle layer
// or the two middle layers (nz alike).  Needs the ghost planes of the state.
__device__ __forceinline__ double centre_density(const Args& a, int x) {
#pragma clang fp contract(off)
  const int y0 = (a.ny - 1) / 2, y1 = a.ny / 2;
  const int z0 = (a.nz - 1) / 2, z1 = a.nz / 2;
  double sum = 0.0;
  int cnt = 0;
  for (int z = z0; z <= z1; ++z)
    for (int y = y0; y <= y1; ++y) {
      double f[27];
      gather<true>(a, x, y, z, f);
      double r, jx, jy, jz;
      rho_j(f, r, jx, jy, jz);
      sum += r;
      ++cnt;
    }
  return sum / (double)cnt;
}

// Relaxation rates of cross-section x of a pressure-driven duct, 32 lanes
// per x, lane i < 27 pulling direction i at the central node(s):
// Kn(x) = Kn_out rho_out / rho_c(x), s_nu(x) by Eq. (18) with N = ny, s_q(x)
// by Eq. (21); the bulk rate stays s_b.  Needs the ghost planes of the state.
__global__ __launch_bounds__(256) void k3_rates(Args a) {
#pragma clang fp contract(off)
  const int i = (int)(threadIdx.x & 31);
  const int e = i % 3 - 1, b = (i / 3) % 3 - 1, c = i / 9 - 1;
  const int y0 = (a.ny - 1) / 2, y1 = a.ny / 2;
  const int z0 = (a.nz - 1) / 2, z1 = a.nz / 2;
  const double cnt = (double)((y1 - y0 + 1) * (z1 - z0 + 1));
  for (size_t g = (blockIdx.x * (size_t)256 + threadIdx.x) >> 5; g < (size_t)a.nx; g += (size_t)gridDim.x * 8) {
    const int x = (int)g;
    double acc = 0.0;
    if (i < 27)
      for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y) acc += pull<true>(a, x, y, z, dev_index(a, x, y, z), e, b, c);
    const double rc = group32_sum(acc) / cnt;
    if (i == 0) {
      double snu, sq;
      clb::local_rates(a.kn, a.rho_out, rc, a.c_tau, a.ab, a.A2, a.tq_den, snu, sq);
      a.col_rates[x] = snu;
      a.col_rates[a.nx + x] = sq;
    }
  }
}

// Mass flow through the cross-sections, first pass: the rows of each
// cross-section are cut into kRowParts contiguous parts; wavefront (x block
// of 64 columns, part r) sums rho u_x (= j_x + rho F_x / 2, Eq. 13) of the
// pre-collision state over its part's rows in order, one column per lane
// (the loads of a row are one 512-byte piece per direction), and writes
// part[r][x].
constexpr int kRowParts = 64;

__global__ __launch_bounds__(64) void k3_mass_parts(Args a, double* part) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * 64 + (int)threadIdx.x;
  if (x >= a.nx) return;
  const size_t cs = (size_t)a.ny * (size_t)a.nz;
  const size_t r = blockIdx.y;
  const size_t k0 = r * cs / kRowParts, k1 = (r + 1) * cs / kRowParts;
  double acc = 0.0;
  for (size_t k = k0; k < k1; ++k) {
    const int y = (int)(k % (size_t)a.ny), z = (int)(k / (size_t)a.ny);
    double f[27];
    gather_any(a, x, y, z, f);
    double rho, jx, jy, jz;
    rho_j(f, rho, jx, jy, jz);
    acc += jx + 0.5 * rho * a.gx;
  }
  part[r * (size_t)a.nx + (size_t)x] = acc;
}

// Second pass, one thread per x: m[x] = the parts in order r = 0, 1, ...
__global__ __launch_bounds__(256) void k3_mass_sum(Args a, const double* __restrict__ part, double* m) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.nx) return;
  double acc = 0.0;
  for (int r = 0; r < kRowParts; ++r) acc += part[(size_t)r * (size_t)a.nx + (size_t)x];
  m[x] = acc;
}

// rhoc[x] = rho_c(x), one thread per x (pressure-driven ducts).
__global__ __launch_bounds__(256) void k3_centre(Args a, double* rhoc) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.nx) return;
  rhoc[x] = centre_density(a, x);
}

// Pressure deviation along the centre line (Section 3.2), one thread per x:
// dp[x] = (p_c(x) - p_l(x)) / p_out, p = rho / 3, p_l linear from p_in at
// x = 0 to p_out at x = nx, node centres at x + 1/2.
__global__ __launch_bounds__(256) void k3_pressure_dev(Args a, const double* __restrict__ rhoc, double* dp) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.nx) return;
  const double p_out = a.rho_out / 3.0, p_in = a.rho_in / 3.0;
  const double p_l = p_in - (p_in - p_out) * ((double)x + 0.5) / (double)a.nx;
  dp[x] = (rhoc[x] / 3.0 - p_l) / p_out;
}

// Count of non-finite values among all populations (logical nodes only: the
// padding lanes of a last row segment are never written), per workgroup.
__global__ __launch_bounds__(256) void k3_nonfinite_partial(const double* __restrict__ p, Args a,
                                                            double* partial) {
  __shared__ double s[4];
  double cnt = 0.0;
  for (size_t n = blockIdx.x * (size_t)256 + threadIdx.x; n < a.plane; n += (size_t)gridDim.x * 256) {
    const int x = (int)(n % (size_t)a.nx);
    const size_t rest = n / (size_t)a.nx;
    const int y = (int)(rest % (size_t)a.ny);
    const int z = (int)(rest / (size_t)a.ny);
    const size_t d = dev_index(a, x, y, z);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const double v = p[((size_t)i << a.lshift) + d];
      cnt += (v - v == 0.0) ? 0.0 : 1.0;   // inf - inf and NaN - NaN are NaN
    }
  }
  cnt = clb::wave_sum(cnt);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Sum of n partials in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k3_sum(const double* __restrict__ v, int n, double* out) {
  __shared__ double s[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
  acc = clb::wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Start: f^eq(rho, 0) (product of the one-axis factors 2/3, 1/6, 1/6) with
// rho = rho0, or falling linearly from rho_in at the inlet plane x = 0 to
// rho_out at the outlet plane x = nx (node centres x + 1/2; kind
// CLB_INIT_LINEAR_RHO), plus the seeded perturbation (CLB_INIT_PERTURBED).
__global__ void k3_init(double* dst, Args a, double rho0, int kind, double amp, uint64_t seed) {
#pragma clang fp contract(off)
  const bool perturbed = kind == CLB_INIT_PERTURBED;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < a.plane; n += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(n % (size_t)a.nx);
    const size_t rest = n / (size_t)a.nx;
    const int y = (int)(rest % (size_t)a.ny);
    const int z = (int)(rest / (size_t)a.ny);
    const size_t d = dev_index(a, x, y, z);
    const double rho = kind == CLB_INIT_LINEAR_RHO
                           ? a.rho_in - (a.rho_in - a.rho_out) * ((double)x + 0.5) / (double)a.nx
                           : rho0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const int e0 = i % 3 - 1, e1 = (i / 3) % 3 - 1, e2 = i / 9 - 1;
      const double w0 = e0 == 0 ? 2.0 / 3.0 : 1.0 / 6.0, w1 = e1 == 0 ? 2.0 / 3.0 : 1.0 / 6.0,
                   w2 = e2 == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
      double v = rho * w0 * w1 * w2;
      if (perturbed) {
        const uint64_t key = seed ^ (27ull * (uint64_t)n + (uint64_t)i);
        const double U = (double)(clb::splitmix64_first(key) >> 11) * (1.0 / 9007199254740992.0);
        v += amp * (2.0 * U - 1.0);
      }
      dst[((size_t)i << a.lshift) + d] = v;
    }
  }
}

// ABI layout [27][nz][ny][nx] <-> device layout.
template <bool EXPORT>
__global__ void k3_convert(const double* __restrict__ src, Args a, double* __restrict__ dst) {
  const size_t n = 27 * a.plane;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(k / a.plane);
    const size_t node = k - (size_t)i * a.plane;
    const int x = (int)(node % (size_t)a.nx);
    const size_t rest = node / (size_t)a.nx;
    const int y = (int)(rest % (size_t)a.ny);
    const int z = (int)(rest / (size_t)a.ny);
    const size_t d = ((size_t)i << a.lshift) + dev_index(a, x, y, z);
    if (EXPORT)
      dst[k] = src[d];
    else
      dst[d] = src[k];
  }
}

constexpr int kPartials = 1024;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workgroups of 256 threads for n groups of 32 lanes (eight per workgroup),
// at most 65536 (the kernels loop over the rest).
unsigned group_blocks(size_t n) {
  size_t b = (n + 7) / 8;
  if (b > 65536) b = 65536;
  return (unsigned)(b == 0 ? 1 : b);
}

unsigned blocks_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > (size_t)kPartials) b = kPartials;
  return (unsigned)(b == 0 ? 1 : b);
}

}  // namespace
}  // namespace clb3

struct clb3_ctx {
  clb3_params p;
  clb_derived d;
  double* buf[2];
  int cur;
  double* partial;
  double* result;
  double* cols;     // [3 + kRowParts][nx]: s_nu(x), s_q(x) of a pressure-driven duct, per-x scratch, mass-flow parts
  double* ghosts;   // [2][nz][ny][27] ghost planes (pressure-driven ducts; NULL otherwise)
  hipStream_t stream;
  int64_t steps;
  // optional hipGraph of graph_steps steps, one per starting buffer
  int graph_steps;
  hipStream_t capture;   // private stream used only to record the graphs
  hipGraph_t graph[2];
  hipGraphExec_t gexec[2];
};

namespace {

constexpr double kPi = 3.14159265358979323846;

clb_status fail3(clb_status st, const char* fmt, ...) {
  char msg[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof(msg), fmt, ap);
  va_end(ap);
  return clb::set_error(st, msg);
}

#define CLB3_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return fail3(CLB_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

bool finite(double v) { return std::isfinite(v); }

clb_status validate3(const clb3_params* p, clb_derived* d) {
  if (!p) return fail3(CLB_EINVAL, "params: NULL");
  if (p->nx < 1) return fail3(CLB_EINVAL, "nx: must be >= 1 (got %d)", p->nx);
  if (p->ny < 1) return fail3(CLB_EINVAL, "ny: must be >= 1 (got %d)", p->ny);
  if (p->nz < 1 || p->nz > 65535) return fail3(CLB_EINVAL, "nz: must lie in [1, 65535] (got %d)", p->nz);
  if ((p->ny + 3) / 4 > 65535) return fail3(CLB_EINVAL, "ny: at most 262140 rows");
  if ((size_t)((p->nx + 63) / 64) * (size_t)((p->ny + 3) / 4) * (size_t)p->nz >= ((size_t)1 << 31))
    return fail3(CLB_EINVAL, "nx*ny*nz: grid too large for one launch");
  if (p->zbc != CLB3_Z_WALLS && p->zbc != CLB3_Z_PERIODIC) return fail3(CLB_EINVAL, "zbc: unknown kind %d", p->zbc);
  if (p->xbc != CLB_X_PERIODIC && p->xbc != CLB_X_PRESSURE) return fail3(CLB_EINVAL, "xbc: unknown kind %d", p->xbc);
  const bool pressure = p->xbc == CLB_X_PRESSURE;
  if (p->init != CLB_INIT_UNIFORM && p->init != CLB_INIT_PERTURBED && p->init != CLB_INIT_LINEAR_RHO)
    return fail3(CLB_EINVAL, "init: unknown kind %d", p->init);
  if (p->init == CLB_INIT_LINEAR_RHO && !pressure)
    return fail3(CLB_EINVAL, "init: CLB_INIT_LINEAR_RHO needs xbc = CLB_X_PRESSURE");
  if (pressure) {
    if (p->nx < 2) return fail3(CLB_EINVAL, "nx: pressure-driven ducts need nx >= 2 (got %d)", p->nx);
    if (p->gx != 0.0 || p->gy != 0.0 || p->gz != 0.0)
      return fail3(CLB_EINVAL, "gx/gy/gz: must be 0 for a pressure-driven duct");
    if (!(finite(p->p_ratio) && p->p_ratio > 0)) return fail3(CLB_EINVAL, "p_ratio: must be finite and > 0");
    if (!(finite(p->rho_out) && p->rho_out > 0)) return fail3(CLB_EINVAL, "rho_out: must be finite and > 0");
    if (!finite(p->p_ratio * p->rho_out)) return fail3(CLB_EINVAL, "p_ratio * rho_out: must be finite");
  }
  if (p->cbbsr_shift != 0 && p->cbbsr_shift != 1) return fail3(CLB_EINVAL, "cbbsr_shift: must be 0 or 1");
  if (p->cbbsr_shift == 0 && p->zbc == CLB3_Z_WALLS)
    return fail3(CLB_EINVAL, "cbbsr_shift: the same-node specular source does not conserve mass at duct edges; "
                             "z-periodic channels only");
  if (!(finite(p->kn) && p->kn > 0)) return fail3(CLB_EINVAL, "kn: must be finite and > 0");
  if (!(finite(p->a) && p->a >= 0)) return fail3(CLB_EINVAL, "a: must be finite and >= 0");
  if (!(finite(p->sigma) && p->sigma > 0 && p->sigma <= 2)) return fail3(CLB_EINVAL, "sigma: must lie in (0, 2]");
  if (!std::isnan(p->A1) && !(finite(p->A1) && p->A1 >= 0))
    return fail3(CLB_EINVAL, "A1: must be NaN (derive from sigma) or finite and >= 0");
  if (!(finite(p->A2) && p->A2 >= 0)) return fail3(CLB_EINVAL, "A2: must be finite and >= 0");
  if (!std::isnan(p->r) && !(p->r >= 0 && p->r <= 1))
    return fail3(CLB_EINVAL, "r: must be NaN (derive from A1) or lie in [0, 1]");
  if (!(finite(p->s_b) && p->s_b > 0 && p->s_b < 2)) return fail3(CLB_EINVAL, "s_b: must lie in (0, 2)");
  if (!(finite(p->s8) && p->s8 > 0 && p->s8 < 2)) return fail3(CLB_EINVAL, "s8: must lie in (0, 2)");
  if (!(finite(p->gx) && finite(p->gy) && finite(p->gz))) return fail3(CLB_EINVAL, "gx/gy/gz: must be finite");
  if (!(finite(p->rho0) && p->rho0 > 0)) return fail3(CLB_EINVAL, "rho0: must be finite and > 0");
  if (!(finite(p->init_amp) && p->init_amp >= 0)) return fail3(CLB_EINVAL, "init_amp: must be finite and >= 0");
  if (!(finite(p->tq_den) && p->tq_den > 0)) return fail3(CLB_EINVAL, "tq_den: must be finite and > 0");
  clb_derived dd;
  dd.A1 = std::isnan(p->A1) ? (1.0 - 0.1817 * p->sigma) * (2.0 - p->sigma) / p->sigma : p->A1;
  dd.r = std::isnan(p->r) ? 1.0 / (1.0 + dd.A1 * std::sqrt(kPi / 6.0)) : p->r;
  dd.tau_tilde = std::sqrt(6.0 / kPi) * (double)p->ny * p->kn / (1.0 + p->a * p->kn);
  dd.s_nu = 1.0 / (0.5 + dd.tau_tilde);
  dd.s_q = 1.0 / (0.5 + (3.0 + 4.0 * kPi * dd.tau_tilde * dd.tau_tilde * p->A2) / (p->tq_den * dd.tau_tilde));
  if (!(dd.s_nu > 0 && dd.s_nu < 2 && dd.s_q > 0 && dd.s_q < 2 && finite(dd.r)))
    return fail3(CLB_EINVAL, "kn/a/A2: derived relaxation rates out of (0, 2)");
  if (d) *d = dd;
  return CLB_OK;
}

size_t plane_of(const clb3_params* p) { return (size_t)p->nx * (size_t)p->ny * (size_t)p->nz; }

// log2 of the row segment length L = min(1024, next power of two >= nx).
int lshift_of(const clb3_params* p) {
  int ls = 0;
  while ((1 << ls) < p->nx && ls < 10) ++ls;
  return ls;
}

int nseg_of(const clb3_params* p) { return (p->nx + (1 << lshift_of(p)) - 1) >> lshift_of(p); }

// One population buffer in the device layout (padded row segments).
size_t buffer_bytes(const clb3_params* p) {
  return clb3::align256((27 * (size_t)p->nz * (size_t)p->ny * (size_t)nseg_of(p) * sizeof(double))
                        << lshift_of(p));
}

// Per-column scratch: s_nu(x), s_q(x), one diagnostic column, the mass
// flow's kRowParts partial columns.
size_t cols_bytes(const clb3_params* p) {
  return clb3::align256((3 + clb3::kRowParts) * (size_t)p->nx * sizeof(double));
}

size_t ghost_bytes(const clb3_params* p) {
  return p->xbc == CLB_X_PRESSURE ? clb3::align256(2 * 27 * (size_t)p->ny * (size_t)p->nz * sizeof(double)) : 0;
}

size_t total_bytes(const clb3_params* p) {
  return 2 * buffer_bytes(p) + clb3::align256(clb3::kPartials * sizeof(double)) + clb3::align256(32 * sizeof(double)) +
         cols_bytes(p) + ghost_bytes(p);
}

// Arguments of a step from buffer cur to the other one.
clb3::Args args_at(const clb3_ctx* c, int cur) {
  clb3::Args a{};
  a.src = c->buf[cur];
  a.dst = c->buf[cur ^ 1];
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.nz = c->p.nz;
  a.lshift = lshift_of(&c->p);
  a.nseg = nseg_of(&c->p);
  a.plane = plane_of(&c->p);
  a.zwalls = c->p.zbc == CLB3_Z_WALLS;
  a.shift = c->p.cbbsr_shift;
  a.r = c->d.r;
  a.omr = 1.0 - c->d.r;
  a.gx = c->p.gx;
  a.gy = c->p.gy;
  a.gz = c->p.gz;
  a.sb = c->p.s_b;
  a.snu = c->d.s_nu;
  a.sq = c->d.s_q;
  a.s8 = c->p.s8;
  a.pressure = c->p.xbc == CLB_X_PRESSURE;
  a.rho_out = c->p.rho_out;
  a.rho_in = c->p.p_ratio * c->p.rho_out;
  a.kn = c->p.kn;
  a.ab = c->p.a;
  a.A2 = c->p.A2;
  a.tq_den = c->p.tq_den;
  a.c_tau = std::sqrt(6.0 / kPi) * (double)c->p.ny;
  a.ghosts = c->ghosts;
  a.col_rates = c->cols;
  return a;
}

clb3::Args args_of(const clb3_ctx* c) { return args_at(c, c->cur); }

// The ghost planes of the state a.src (pressure-driven ducts) on stream st:
// the step, and every diagnostic that gathers, reads them.
void launch_ghosts(const clb3_ctx* c, const clb3::Args& a, hipStream_t st) {
  clb3::k3_ghosts<<<clb3::group_blocks(2 * (size_t)c->p.ny * (size_t)c->p.nz), 256, 0, st>>>(a);
}

clb_status refresh_ghosts(clb3_ctx* c, const clb3::Args& a) {
  if (!a.pressure) return CLB_OK;
  launch_ghosts(c, a, c->stream);
  CLB3_HIP(hipGetLastError());
  return CLB_OK;
}

dim3 node_grid(const clb3_params* p);

// Enqueue n steps on stream st starting from buffer parity *cur (updated
// per step enqueued): per step of a pressure-driven duct the ghost planes,
// the rates of every cross-section and the step; otherwise the step alone.
// *done counts the steps enqueued (all n unless a launch fails).
hipError_t enqueue_steps3(const clb3_ctx* c, int64_t n, hipStream_t st, int* cur, int64_t* done) {
  *done = 0;
  const dim3 g3 = node_grid(&c->p);
  const dim3 grid(g3.x * g3.y * g3.z);   // k3_step orders its workgroups itself
  const bool force = c->p.gx != 0.0 || c->p.gy != 0.0 || c->p.gz != 0.0;
  const bool pressure = c->p.xbc == CLB_X_PRESSURE;
  for (int64_t k = 0; k < n; ++k) {
    const clb3::Args a = args_at(c, *cur);
    if (pressure) {
      launch_ghosts(c, a, st);
      clb3::k3_rates<<<clb3::group_blocks((size_t)c->p.nx), 256, 0, st>>>(a);
      clb3::k3_step<false, true><<<grid, clb3::kBX * clb3::kBY, 0, st>>>(a);
    } else if (force) {
      clb3::k3_step<true, false><<<grid, clb3::kBX * clb3::kBY, 0, st>>>(a);
    } else {
      clb3::k3_step<false, false><<<grid, clb3::kBX * clb3::kBY, 0, st>>>(a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    *cur ^= 1;
    *done += 1;
  }
  return hipSuccess;
}

void drop_graphs3(clb3_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
}

// Record graph_steps steps starting from buffer parity c->cur on the
// private capture stream (recording only: nothing runs there).
clb_status record_graph3(clb3_ctx* c) {
  const int p = c->cur;
  if (!c->capture) CLB3_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  CLB3_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
  int cur = p;
  int64_t done = 0;
  const hipError_t e = enqueue_steps3(c, c->graph_steps, c->capture, &cur, &done);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->capture, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail3(CLB_EHIP, "step launch during graph capture: %s", hipGetErrorString(e));
  }
  if (e2 != hipSuccess) return fail3(CLB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
  c->graph[p] = g;
  CLB3_HIP(hipGraphInstantiate(&c->gexec[p], g, nullptr, nullptr, 0));
  return CLB_OK;
}

dim3 node_grid(const clb3_params* p) {
  return dim3((unsigned)((p->nx + clb3::kBX - 1) / clb3::kBX), (unsigned)((p->ny + clb3::kBY - 1) / clb3::kBY),
              (unsigned)p->nz);
}

clb_status read_result3(clb3_ctx* c, double* h) {
  CLB3_HIP(hipMemcpyAsync(h, c->result, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CLB3_HIP(hipStreamSynchronize(c->stream));
  return CLB_OK;
}

}  // namespace

extern "C" {

void clb3_params_default(clb3_params* p) {
  if (!p) return;
  *p = clb3_params{};
  p->nx = p->ny = p->nz = 1;
  p->zbc = CLB3_Z_WALLS;
  p->init = CLB_INIT_UNIFORM;
  p->cbbsr_shift = 1;
  p->kn = 0.1;
  p->a = 2.0;       // Section 3
  p->sigma = 1.0;
  p->A1 = NAN;
  p->A2 = 0.55;     // Section 3
  p->r = NAN;
  p->s_b = 1.1;     // the paper's s3
  p->s8 = 1.2;      // Section 3
  p->rho0 = 1.0;
  p->tq_den = 16.0;
  p->xbc = CLB_X_PERIODIC;
  p->p_ratio = 2.0;   // Section 3.2
  p->rho_out = 1.0;
}

clb_status clb3_derive(const clb3_params* p, clb_derived* out) {
  if (!out) return fail3(CLB_EINVAL, "out: NULL");
  return validate3(p, out);
}

clb_status clb3_workspace_size(const clb3_params* p, size_t* bytes) {
  if (!bytes) return fail3(CLB_EINVAL, "bytes: NULL");
  clb_status st = validate3(p, nullptr);
  if (st != CLB_OK) return st;
  *bytes = total_bytes(p);
  return CLB_OK;
}

clb_status clb3_init(const clb3_params* p, void* d_workspace, size_t bytes, void* hip_stream, clb3_ctx** out) {
  const clb::TraceRange trace("clb3_init");
  if (!out) return fail3(CLB_EINVAL, "out: NULL");
  *out = nullptr;
  clb_derived d;
  clb_status st = validate3(p, &d);
  if (st != CLB_OK) return st;
  const size_t need = total_bytes(p);
  if (!d_workspace) return fail3(CLB_EINVAL, "d_workspace: NULL");
  if (bytes < need) return fail3(CLB_ENOMEM, "workspace: %zu bytes given, %zu needed", bytes, need);
  if ((st = clb::check_device_ptr(d_workspace, need, "d_workspace")) != CLB_OK) return st;
  clb3_ctx* c = new (std::nothrow) clb3_ctx();
  if (!c) return fail3(CLB_ENOMEM, "host context allocation failed");
  c->p = *p;
  c->d = d;
  char* base = static_cast<char*>(d_workspace);
  c->buf[0] = reinterpret_cast<double*>(base);
  c->buf[1] = reinterpret_cast<double*>(base + buffer_bytes(p));
  c->partial = reinterpret_cast<double*>(base + 2 * buffer_bytes(p));
  c->result = c->partial + clb3::kPartials;
  char* tail = base + 2 * buffer_bytes(p) + clb3::align256(clb3::kPartials * sizeof(double)) +
               clb3::align256(32 * sizeof(double));
  c->cols = reinterpret_cast<double*>(tail);
  c->ghosts = p->xbc == CLB_X_PRESSURE ? reinterpret_cast<double*>(tail + cols_bytes(p)) : nullptr;
  c->cur = 0;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  const size_t plane = plane_of(p);
  clb3::k3_init<<<clb3::blocks_for(plane) * 16, 256, 0, c->stream>>>(c->buf[0], args_of(c), p->rho0, p->init,
                                                                     p->init_amp, p->seed);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete c;
    return fail3(CLB_EHIP, "clb3_init: init kernel: %s", hipGetErrorString(e));
  }
  *out = c;
  return CLB_OK;
}

clb_status clb3_step(clb3_ctx* c, int64_t nsteps) {
  const clb::TraceRange trace("clb3_step");
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (nsteps < 0) return fail3(CLB_EINVAL, "nsteps: must be >= 0");
  clb_status st = CLB_OK;
  while (c->graph_steps > 0 && nsteps >= c->graph_steps) {
    if (!c->gexec[c->cur] && (st = record_graph3(c)) != CLB_OK) return st;
    CLB3_HIP(hipGraphLaunch(c->gexec[c->cur], c->stream));
    c->cur ^= c->graph_steps & 1;   // every step swaps the buffers
    c->steps += c->graph_steps;
    nsteps -= c->graph_steps;
  }
  int64_t done = 0;
  const hipError_t e = enqueue_steps3(c, nsteps, c->stream, &c->cur, &done);
  c->steps += done;
  if (e != hipSuccess) return fail3(CLB_EHIP, "clb3_step: %s", hipGetErrorString(e));
  return CLB_OK;
}

clb_status clb3_set_graph_steps(clb3_ctx* c, int32_t steps_per_graph) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (steps_per_graph < 0 || steps_per_graph > 100000)
    return fail3(CLB_EINVAL, "steps_per_graph: must lie in [0, 100000]");
  if (steps_per_graph != c->graph_steps) {
    CLB3_HIP(hipStreamSynchronize(c->stream));
    drop_graphs3(c);
    c->graph_steps = steps_per_graph;
  }
  return CLB_OK;
}

clb_status clb3_steps_done(const clb3_ctx* c, int64_t* h_steps) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (!h_steps) return fail3(CLB_EINVAL, "h_steps: NULL");
  *h_steps = c->steps;
  return CLB_OK;
}

clb_status clb3_moments(clb3_ctx* c, double* d_rho, double* d_ux, double* d_uy, double* d_uz) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  const size_t bytes = plane_of(&c->p) * sizeof(double);
  clb_status st;
  if (d_rho && (st = clb::check_device_ptr(d_rho, bytes, "d_rho")) != CLB_OK) return st;
  if (d_ux && (st = clb::check_device_ptr(d_ux, bytes, "d_ux")) != CLB_OK) return st;
  if (d_uy && (st = clb::check_device_ptr(d_uy, bytes, "d_uy")) != CLB_OK) return st;
  if (d_uz && (st = clb::check_device_ptr(d_uz, bytes, "d_uz")) != CLB_OK) return st;
  if (!d_rho && !d_ux && !d_uy && !d_uz) return CLB_OK;
  const clb3::Args a = args_of(c);
  if ((st = refresh_ghosts(c, a)) != CLB_OK) return st;
  clb3::k3_moments<<<node_grid(&c->p), clb3::kBX * clb3::kBY, 0, c->stream>>>(a, d_rho, d_ux, d_uy, d_uz);
  CLB3_HIP(hipGetLastError());
  return CLB_OK;
}

clb_status clb3_massflow(clb3_ctx* c, double* d_m_col, double* h_m_mean) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  clb_status st;
  if (d_m_col && (st = clb::check_device_ptr(d_m_col, (size_t)c->p.nx * sizeof(double), "d_m_col")) != CLB_OK)
    return st;
  if (!d_m_col && !h_m_mean) return CLB_OK;
  const clb3::Args a = args_of(c);
  if ((st = refresh_ghosts(c, a)) != CLB_OK) return st;
  double* m = d_m_col ? d_m_col : c->cols + 2 * (size_t)c->p.nx;
  double* part = c->cols + 3 * (size_t)c->p.nx;
  clb3::k3_mass_parts<<<dim3((unsigned)((c->p.nx + 63) / 64), clb3::kRowParts), 64, 0, c->stream>>>(a, part);
  clb3::k3_mass_sum<<<(unsigned)((c->p.nx + 255) / 256), 256, 0, c->stream>>>(a, part, m);
  CLB3_HIP(hipGetLastError());
  if (!h_m_mean) return CLB_OK;
  clb3::k3_sum<<<1, 256, 0, c->stream>>>(m, c->p.nx, c->result);
  CLB3_HIP(hipGetLastError());
  double sum = 0;
  if ((st = read_result3(c, &sum)) != CLB_OK) return st;
  *h_m_mean = sum / (double)c->p.nx;
  return CLB_OK;
}

clb_status clb3_pressure_deviation(clb3_ctx* c, double* d_dp, double* d_rho_c) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (c->p.xbc != CLB_X_PRESSURE) return fail3(CLB_ESTATE, "clb3_pressure_deviation: pressure-driven ducts only");
  const size_t bytes = (size_t)c->p.nx * sizeof(double);
  clb_status st;
  if (d_dp && (st = clb::check_device_ptr(d_dp, bytes, "d_dp")) != CLB_OK) return st;
  if (d_rho_c && (st = clb::check_device_ptr(d_rho_c, bytes, "d_rho_c")) != CLB_OK) return st;
  if (!d_dp && !d_rho_c) return CLB_OK;
  const clb3::Args a = args_of(c);
  if ((st = refresh_ghosts(c, a)) != CLB_OK) return st;
  double* rc = d_rho_c ? d_rho_c : c->cols + 2 * (size_t)c->p.nx;
  clb3::k3_centre<<<(unsigned)((c->p.nx + 255) / 256), 256, 0, c->stream>>>(a, rc);
  if (d_dp) clb3::k3_pressure_dev<<<(unsigned)((c->p.nx + 255) / 256), 256, 0, c->stream>>>(a, rc, d_dp);
  CLB3_HIP(hipGetLastError());
  return CLB_OK;
}

clb_status clb3_flow_rate(clb3_ctx* c, double* h_Q) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (!h_Q) return fail3(CLB_EINVAL, "h_Q: NULL");
  if (c->p.gx == 0) return fail3(CLB_ESTATE, "clb3_flow_rate: needs gx != 0");
  const unsigned nb = clb3::blocks_for(plane_of(&c->p));
  clb3::k3_ux_partial<<<nb, 256, 0, c->stream>>>(args_of(c), c->partial);
  clb3::k3_sum<<<1, 256, 0, c->stream>>>(c->partial, (int)nb, c->result);
  CLB3_HIP(hipGetLastError());
  double su = 0;
  clb_status st = read_result3(c, &su);
  if (st != CLB_OK) return st;
  const double H = (double)c->p.ny, W = (double)c->p.nz;
  *h_Q = (su / (double)c->p.nx) * std::sqrt(6.0) / (3.0 * c->p.gx * H * H * W);
  return CLB_OK;
}

clb_status clb3_get_populations(clb3_ctx* c, double* d_out) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  const size_t bytes = 27 * plane_of(&c->p) * sizeof(double);
  clb_status st = clb::check_device_ptr(d_out, bytes, "d_out");
  if (st != CLB_OK) return st;
  clb3::k3_convert<true><<<clb3::blocks_for(27 * plane_of(&c->p)) * 16, 256, 0, c->stream>>>(c->buf[c->cur],
                                                                                            args_of(c), d_out);
  CLB3_HIP(hipGetLastError());
  return CLB_OK;
}

clb_status clb3_set_populations(clb3_ctx* c, const double* d_in) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  const size_t bytes = 27 * plane_of(&c->p) * sizeof(double);
  clb_status st = clb::check_device_ptr(d_in, bytes, "d_in");
  if (st != CLB_OK) return st;
  clb3::k3_convert<false><<<clb3::blocks_for(27 * plane_of(&c->p)) * 16, 256, 0, c->stream>>>(d_in, args_of(c),
                                                                                             c->buf[c->cur]);
  CLB3_HIP(hipGetLastError());
  c->steps = 0;
  return CLB_OK;
}

clb_status clb3_check_finite(clb3_ctx* c, int32_t* h_ok) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (!h_ok) return fail3(CLB_EINVAL, "h_ok: NULL");
  const unsigned nb = clb3::blocks_for(plane_of(&c->p));
  clb3::k3_nonfinite_partial<<<nb, 256, 0, c->stream>>>(c->buf[c->cur], args_of(c), c->partial);
  clb3::k3_sum<<<1, 256, 0, c->stream>>>(c->partial, (int)nb, c->result);
  CLB3_HIP(hipGetLastError());
  double bad = 0;
  clb_status st = read_result3(c, &bad);
  if (st != CLB_OK) return st;
  *h_ok = bad == 0.0 ? 1 : 0;
  if (!*h_ok) return fail3(CLB_EUNSTABLE, "populations: %.0f non-finite values", bad);
  return CLB_OK;
}

clb_status clb3_destroy(clb3_ctx* c) {
  if (!c) return fail3(CLB_EINVAL, "ctx: NULL");
  if (c->gexec[0] || c->gexec[1]) (void)hipStreamSynchronize(c->stream);
  drop_graphs3(c);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
  return CLB_OK;
}

}  // extern "C"
