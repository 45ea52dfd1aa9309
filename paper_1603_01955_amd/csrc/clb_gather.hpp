// Pull-streaming gather of the pre-collision populations of one node, with
// the CBBSR walls and the x boundaries (shared by every step kernel).
//
// Method: Liu & He, arXiv:1603.01955, Eq. (5) (streaming), Eq. (20) (walls),
// Sections 3.1-3.2 (periodic and pressure inlet/outlet).
#pragma once

#include "clb_device.hpp"
#include "clb_internal.hpp"

namespace clb {
namespace {

// ---------------------------------------------------------------------------
// Gather of the pre-collision populations of node (x, y).
// MODE 0: periodic x.  MODE 1: pressure ghost columns at x = -1 and x = nx.
// ---------------------------------------------------------------------------
// Populations in the device layout of a single-channel buffer (HBM).
struct View {
  const double* __restrict__ P;
  Geo g;
  __device__ __forceinline__ double at(int i, int x, int y) const { return P[g.index(i, x, y)]; }
  __device__ __forceinline__ int nx() const { return g.nx; }
  __device__ __forceinline__ int ny() const { return g.ny; }
};

// Populations of one channel held in LDS, plane layout [9][ny][nx].
struct LdsView {
  const double* P;
  int nx_, ny_, n;
  __device__ __forceinline__ double at(int i, int x, int y) const { return P[i * n + y * nx_ + x]; }
  __device__ __forceinline__ int nx() const { return nx_; }
  __device__ __forceinline__ int ny() const { return ny_; }
};

// The nine populations of a pressure ghost column at row y.  Reading adopted
// for the extrapolation scheme the paper cites (Section 3.2): density
// extrapolated so that the boundary plane carries rho_b, velocity
// extrapolated linearly from the two adjacent columns, non-equilibrium part
// copied from the adjacent column:
//   f_g = f^eq(2 rho_b - rho_1, 2 u_1 - u_2) + f_1 - f^eq(rho_1, u_1).
template <class V>
__device__ __forceinline__ void ghost_row(const V& v, bool inlet, int y, double rho_b, double g[9]) {
#pragma clang fp contract(off)
  const int c1 = inlet ? 0 : v.nx() - 1;
  const int c2 = inlet ? 1 : v.nx() - 2;
  double f1[9], f2[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    f1[k] = v.at(k, c1, y);
    f2[k] = v.at(k, c2, y);
  }
  double rho1, ux1, uy1, rho2, ux2, uy2;
  rho_u(f1, rho1, ux1, uy1);
  rho_u(f2, rho2, ux2, uy2);
  double eg[9], e1[9];
  equilibrium(2.0 * rho_b - rho1, 2.0 * ux1 - ux2, 2.0 * uy1 - uy2, eg);
  equilibrium(rho1, ux1, uy1, e1);
#pragma unroll
  for (int k = 0; k < 9; ++k) g[k] = eg[k] + (f1[k] - e1[k]);
}

// Population i of a ghost column, evaluated on the spot.
template <class V>
__device__ __noinline__ double ghost_pop(V v, bool inlet, int y, double rho_b, int i) {
  double g[9];
  ghost_row(v, inlet, y, rho_b, g);
  double out = g[0];
#pragma unroll
  for (int k = 1; k < 9; ++k)
    if (k == i) out = g[k];
  return out;
}

// Largest ny whose two ghost columns ([2][9][ny] doubles) are staged in LDS.
constexpr int kGhostLdsMaxNy = 512;

// The workgroups at the inlet / outlet build the ghost columns they read once
// per step, one row per thread, into s_in / s_out ([9][ny] each).
template <class V>
__device__ __forceinline__ void fill_ghosts(const V& v, double rho_in, double rho_out, bool need_in, bool need_out,
                                            double* s_in, double* s_out, int tid, int nthreads) {
  const int ny = v.ny();
  for (int y = tid; y < ny; y += nthreads) {
    double g[9];
    if (need_in) {
      ghost_row(v, true, y, rho_in, g);
#pragma unroll
      for (int k = 0; k < 9; ++k) s_in[k * ny + y] = g[k];
    }
    if (need_out) {
      ghost_row(v, false, y, rho_out, g);
#pragma unroll
      for (int k = 0; k < 9; ++k) s_out[k * ny + y] = g[k];
    }
  }
}

template <int MODE, class V>
struct Gather {
  V v;
  double r, omr;        // bounce-back fraction r and 1 - r (Eq. 20)
  int shift;            // specular source from x -/+ 1 (1) or the same node (0)
  double rho_in, rho_out;
  // Optional precomputed ghost columns [9][ny] (LDS) for x = -1 and x = nx;
  // when null the ghost population is evaluated on the spot.
  const double* gin = nullptr;
  const double* gout = nullptr;

  // P_i at column xs (possibly -1 or nx) and row ys (always inside).
  __device__ __forceinline__ double pop(int i, int xs, int ys) const {
    if (MODE == 0) {
      if (xs < 0) xs += v.nx();
      else if (xs >= v.nx()) xs -= v.nx();
      return v.at(i, xs, ys);
    } else {
      if (xs < 0) return gin ? gin[i * v.ny() + ys] : ghost_pop(v, true, ys, rho_in, i);
      if (xs >= v.nx()) return gout ? gout[i * v.ny() + ys] : ghost_pop(v, false, ys, rho_out, i);
      return v.at(i, xs, ys);
    }
  }

  __device__ __forceinline__ void operator()(int x, int y, double f[9]) const {
#pragma clang fp contract(off)
    f[0] = pop(0, x, y);
    f[1] = pop(1, x - 1, y);
    f[3] = pop(3, x + 1, y);
    const int xsm = shift ? x - 1 : x;
    const int xsp = shift ? x + 1 : x;
    if (y > 0) {
      f[2] = pop(2, x, y - 1);
      f[5] = pop(5, x - 1, y - 1);
      f[6] = pop(6, x + 1, y - 1);
    } else {  // bottom wall, Eq. (20)
      f[2] = pop(4, x, 0);
      f[5] = r * pop(7, x, 0) + omr * pop(8, xsm, 0);
      f[6] = r * pop(8, x, 0) + omr * pop(7, xsp, 0);
    }
    const int t = v.ny() - 1;
    if (y < t) {
      f[4] = pop(4, x, y + 1);
      f[7] = pop(7, x + 1, y + 1);
      f[8] = pop(8, x - 1, y + 1);
    } else {  // top wall: mirror image of Eq. (20)
      f[4] = pop(2, x, t);
      f[7] = r * pop(5, x, t) + omr * pop(6, xsp, t);
      f[8] = r * pop(6, x, t) + omr * pop(5, xsm, t);
    }
  }
};

}  // namespace
}  // namespace clb
