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

// Block index with optional XCD-aware remap: blocks are dealt to the 8 XCDs
// round-robin, so logical block (xcd * per + k) makes each XCD walk a
// contiguous run of row segments or columns (cache lines shared by
// neighbouring workgroups stay in one L2).
__device__ __forceinline__ int logical_block(int remap) {
  int b = blockIdx.x;
  if (remap) {
    const int nb = gridDim.x;
    const int per = nb >> 3;
    if (b < (per << 3)) b = (b & 7) * per + (b >> 3);
  }
  return b;
}

// ---------------------------------------------------------------------------
// Gather of the pre-collision populations of node (x, y).
// MODE 0: periodic x.
// MODE 1: pressure ghost columns at x = -1 and x = nx; the nodes of the first
//         and last column evaluate the ghost populations they pull inline.
// MODE 2: pressure ghost columns read from precomputed arrays gin, gout
//         ([9][ny] each, in LDS or global memory).
// MODE 3: a node whose x - 1 and x + 1 both lie inside the grid (interior
//         workgroups of the pressure kernels): no x-boundary code at all.
// ---------------------------------------------------------------------------
// Populations in the device layout of a single-channel buffer (HBM).
struct View {
  const double* __restrict__ P;
  Geo g;
  __device__ __forceinline__ double at(int i, int x, int y) const { return P[g.index(i, x, y)]; }
  __device__ __forceinline__ const double* ptr(int i, int x, int y) const { return P + g.index(i, x, y); }
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

// Populations in the ABI layout [9][ny][nx] (x fastest) in device memory.
struct PlaneView {
  const double* __restrict__ P;
  int nx_, ny_;
  __device__ __forceinline__ const double* ptr(int i, int x, int y) const {
    return P + ((size_t)i * (size_t)ny_ + (size_t)y) * (size_t)nx_ + (size_t)x;
  }
  __device__ __forceinline__ double at(int i, int x, int y) const { return *ptr(i, x, y); }
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

// One factor of the product-form equilibrium (as in `equilibrium`) for a
// velocity component e = -1, 0, +1.
__device__ __forceinline__ double eq_factor(int e, double u) {
#pragma clang fp contract(off)
  return e == 0 ? 2.0 / 3.0 - u * u : (e > 0 ? 0.5 * (1.0 / 3.0 + u * u + u) : 0.5 * (1.0 / 3.0 + u * u - u));
}

// Ghost population i from the density and velocity of the two adjacent
// columns (rho1, u1 next to the boundary, u2 one further in) and the
// adjacent column's own population f1i: ghost_row's arithmetic for that one
// direction (bitwise the same value).
__device__ __forceinline__ double ghost_from(int i, double rho_b, double rho1, double ux1, double uy1, double ux2,
                                             double uy2, double f1i) {
#pragma clang fp contract(off)
  const int ex = (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
  const int ey = (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
  const double eg = (2.0 * rho_b - rho1) * eq_factor(ex, 2.0 * ux1 - ux2) * eq_factor(ey, 2.0 * uy1 - uy2);
  const double e1 = rho1 * eq_factor(ex, ux1) * eq_factor(ey, uy1);
  return eg + (f1i - e1);
}

// Population i of the ghost column at row y, evaluated inline.
template <class V>
__device__ __forceinline__ double ghost_value(const V& v, bool inlet, int y, double rho_b, int i) {
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
  double f1i = f1[0];
#pragma unroll
  for (int k = 1; k < 9; ++k) f1i = k == i ? f1[k] : f1i;
  return ghost_from(i, rho_b, rho1, ux1, uy1, ux2, uy2, f1i);
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

// fill_ghosts with a smaller register footprint, for kernels that keep
// many waves in flight: one thread per row takes the velocity of the second
// column, then the first column's populations and moments, and writes the
// nine ghost populations one by one (bitwise ghost_row's values).  No
// barrier: the caller synchronises before the ghosts are read.
template <class V>
__device__ __forceinline__ void fill_ghosts_lean(const V& v, double rho_in, double rho_out, bool need_in,
                                                 bool need_out, double* s_in, double* s_out, int tid, int nthreads) {
  const int ny = v.ny(), nx = v.nx();
  for (int j = tid; j < 2 * ny; j += nthreads) {
    const bool inlet = j < ny;
    if (inlet ? !need_in : !need_out) continue;
    const int y = inlet ? j : j - ny;
    const int c1 = inlet ? 0 : nx - 1, c2 = inlet ? 1 : nx - 2;
    double f[9], rho1, ux1, uy1, rho2, ux2, uy2;
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = v.at(k, c2, y);
    rho_u(f, rho2, ux2, uy2);
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = v.at(k, c1, y);
    rho_u(f, rho1, ux1, uy1);
    double* out = inlet ? s_in : s_out;
    const double rho_b = inlet ? rho_in : rho_out;
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i * ny + y] = ghost_from(i, rho_b, rho1, ux1, uy1, ux2, uy2, f[i]);
  }
}

template <int MODE, class V>
struct Gather {
  V v;
  double r, omr;        // bounce-back fraction r and 1 - r (Eq. 20)
  int shift;            // specular source from x -/+ 1 (1) or the same node (0)
  double rho_in, rho_out;
  // MODE 2: ghost columns [9][ny] for x = -1 and x = nx.
  const double* gin = nullptr;
  const double* gout = nullptr;

  // P_i at column xs (possibly -1 or nx) and row ys (always inside).
  __device__ __forceinline__ double pop(int i, int xs, int ys) const {
    if (MODE == 0) {
      if (xs < 0) xs += v.nx();
      else if (xs >= v.nx()) xs -= v.nx();
    } else if (MODE == 1) {
      if (xs < 0) return ghost_value(v, true, ys, rho_in, i);
      if (xs >= v.nx()) return ghost_value(v, false, ys, rho_out, i);
    } else if (MODE == 2) {
      if (xs < 0) return gin[i * v.ny() + ys];
      if (xs >= v.nx()) return gout[i * v.ny() + ys];
    }
    return v.at(i, xs, ys);
  }

  // Branch-free form (MODES 1-3): every source address is selected first
  // and all loads issue together, so a wave waits on memory once.
  // A[i] is the population pulled into direction i, or for a wall-replaced
  // direction its bounce-back part; B[k] (k = 0..3 for directions 5..8) is
  // the specular part (Eq. 20), a duplicate of A's address off the walls.
  // MODE 2 addresses a ghost source in gin / gout directly.  With CLAMP
  // (always for MODE 1) a ghost source is loaded from a clamped in-grid
  // address instead and its value replaced afterwards (patch_ghosts), so the
  // loads can be issued before the ghost values exist.
  template <bool CLAMP>
  __device__ __forceinline__ const double* addr(int i, int xs, int ys) const {
    static_assert(MODE >= 1 && MODE <= 3, "addresses exist for the pressure modes only");
    if (MODE == 3) return v.ptr(i, xs, ys);
    const int xc = xs < 0 ? 0 : (xs >= v.nx() ? v.nx() - 1 : xs);
    const double* p = v.ptr(i, xc, ys);
    if (MODE == 2 && !CLAMP) {
      p = xs < 0 ? gin + i * v.ny() + ys : p;
      p = xs >= v.nx() ? gout + i * v.ny() + ys : p;
    }
    return p;
  }

  // Population i of ghost row ys (inlet or outlet side).
  __device__ __forceinline__ double ghost(bool inlet, int ys, int i) const {
    if (MODE == 2) return (inlet ? gin : gout)[i * v.ny() + ys];
    return ghost_value(v, inlet, ys, inlet ? rho_in : rho_out, i);
  }

  __device__ __forceinline__ void sources(int x, int y, double A[9], double B[4]) const {
    load_sources<MODE == 1>(x, y, A, B);
    if (MODE == 1) patch_ghosts(x, y, A, B);
  }

  template <bool CLAMP>
  __device__ __forceinline__ void load_sources(int x, int y, double A[9], double B[4]) const {
    const int t = v.ny() - 1;
    const bool bot = y == 0, top = y == t;
    const int ym = bot ? 0 : y - 1, yp = top ? t : y + 1;
    const int xsm = shift ? x - 1 : x;
    const int xsp = shift ? x + 1 : x;
    const double* a[9];
    const double* b[4];
    a[0] = addr<CLAMP>(0, x, y);
    a[1] = addr<CLAMP>(1, x - 1, y);
    a[3] = addr<CLAMP>(3, x + 1, y);
    a[2] = bot ? addr<CLAMP>(4, x, 0) : addr<CLAMP>(2, x, ym);
    a[5] = bot ? addr<CLAMP>(7, x, 0) : addr<CLAMP>(5, x - 1, ym);
    a[6] = bot ? addr<CLAMP>(8, x, 0) : addr<CLAMP>(6, x + 1, ym);
    a[4] = top ? addr<CLAMP>(2, x, t) : addr<CLAMP>(4, x, yp);
    a[7] = top ? addr<CLAMP>(5, x, t) : addr<CLAMP>(7, x + 1, yp);
    a[8] = top ? addr<CLAMP>(6, x, t) : addr<CLAMP>(8, x - 1, yp);
    b[0] = bot ? addr<CLAMP>(8, xsm, 0) : a[5];
    b[1] = bot ? addr<CLAMP>(7, xsp, 0) : a[6];
    b[2] = top ? addr<CLAMP>(6, xsp, t) : a[7];
    b[3] = top ? addr<CLAMP>(5, xsm, t) : a[8];
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i] = *a[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) B[k] = *b[k];
  }

  // The ghost populations node (x, y) pulls (MODES 1, 2).  A first-column node
  // pulls direction 1 from ghost row y, 5 from row y - 1 and 8 from row
  // y + 1; on a wall row the ghost enters as the specular partner instead
  // (8 at the bottom, 5 at the top, when the source is shifted).  The last
  // column mirrors this with 3, 6, 7.
  __device__ __forceinline__ void patch_ghosts(int x, int y, double A[9], double B[4]) const {
    const int t = v.ny() - 1;
    const bool bot = y == 0, top = y == t;
    const int rlo = bot ? 0 : y - 1, rhi = top ? t : y + 1;
    if (x == 0) {
      const double gm = ghost(true, y, 1);
      const double gl = ghost(true, rlo, bot ? 8 : 5);
      const double gh = ghost(true, rhi, top ? 5 : 8);
      A[1] = gm;
      if (!bot) A[5] = gl;
      else if (shift) B[0] = gl;
      if (!top) A[8] = gh;
      else if (shift) B[3] = gh;
    }
    if (x == v.nx() - 1) {
      const double gm = ghost(false, y, 3);
      const double gl = ghost(false, rlo, bot ? 7 : 6);
      const double gh = ghost(false, rhi, top ? 6 : 7);
      A[3] = gm;
      if (!bot) A[6] = gl;
      else if (shift) B[1] = gl;
      if (!top) A[7] = gh;
      else if (shift) B[2] = gh;
    }
  }

  __device__ __forceinline__ void combine(int y, const double A[9], const double B[4], double f[9]) const {
#pragma clang fp contract(off)
    const bool bot = y == 0, top = y == v.ny() - 1;
#pragma unroll
    for (int i = 0; i < 5; ++i) f[i] = A[i];
    f[5] = bot ? r * A[5] + omr * B[0] : A[5];
    f[6] = bot ? r * A[6] + omr * B[1] : A[6];
    f[7] = top ? r * A[7] + omr * B[2] : A[7];
    f[8] = top ? r * A[8] + omr * B[3] : A[8];
  }

  // lp . d pre / d r of a wall node from its sources (Eq. 20); 0 off the walls.
  __device__ __forceinline__ double wall_dr(int y, const double A[9], const double B[4], const double lp[9]) const {
#pragma clang fp contract(off)
    double dr = 0.0;
    if (y == 0) {
      dr += lp[5] * (A[5] - B[0]);
      dr += lp[6] * (A[6] - B[1]);
    }
    if (y == v.ny() - 1) {
      dr += lp[7] * (A[7] - B[2]);
      dr += lp[8] * (A[8] - B[3]);
    }
    return dr;
  }

  __device__ __forceinline__ void flat(int x, int y, double f[9]) const {
    double A[9], B[4];
    sources(x, y, A, B);
    combine(y, A, B, f);
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

// The gather of one node in the best form the mode allows.
template <int MODE, class V>
__device__ __forceinline__ void gather_node(const Gather<MODE, V>& g, int x, int y, double f[9]) {
  if constexpr (MODE >= 1)
    g.flat(x, y, f);
  else
    g(x, y, f);
}

}  // namespace
}  // namespace clb
