// HIP kernels of the D2Q9 cascaded LB step for gfx950 (MI355X).
//
// Method: Liu & He, arXiv:1603.01955.  Streaming (Eq. 5) is done as a pull:
// node (x, y) reads P_i from (x - e_ix, y - e_iy), except where that source
// lies behind a wall (Eq. 20, half-way walls below row 0 and above row
// ny - 1) or outside the inlet/outlet (periodic wrap, Section 3.1, or
// pressure ghost columns, Section 3.2).  A step is one fused kernel:
// gather -> cascaded collision (Eqs. 4, 6-9, 13) -> store to the other
// buffer, so each node update moves 72 B in and 72 B out of HBM.  The
// multi-step kernels (K1b periodic, K2e pressure) keep the steps before the
// last in LDS, computed over a halo of the workgroup's tile, and move about
// half of that per node update.
#include "clb_device.hpp"
#include "clb_gather.hpp"
#include "clb_internal.hpp"

namespace clb {

Geo make_geo(int nx, int ny) {
  Geo g;
  g.nx = nx;
  g.ny = ny;
  int ls = 0;
  while ((1 << ls) < nx && ls < 10) ++ls;   // L = min(1024, next power of two >= nx)
  g.lshift = ls;
  g.nseg = (nx + (1 << ls) - 1) >> ls;
  return g;
}

namespace {

__device__ __forceinline__ void store9(double* __restrict__ Q, const Geo& g, int x, int y, const double f[9]) {
  const size_t base = g.index(0, x, y);
  const size_t stride = (size_t)1 << g.lshift;
#pragma unroll
  for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(f[i], Q + base + (size_t)i * stride);
}

// ---------------------------------------------------------------------------
// K1: fused periodic step.  One thread per node; threads enumerate the
// padded nodes in device-layout order (y, segment, lane).
// ---------------------------------------------------------------------------
template <bool FORCE, bool THIRD>
__global__ __launch_bounds__(1024) void k_step_periodic(StepArgs a) {
  const size_t t = (size_t)logical_block(a.xcd_remap) * blockDim.x + threadIdx.x;
  const int lane = (int)(t & (((size_t)1 << a.g.lshift) - 1));
  const size_t rest = t >> a.g.lshift;
  const int y = (int)(rest / (size_t)a.g.nseg);
  const int x = (int)(rest - (size_t)y * a.g.nseg) * (1 << a.g.lshift) + lane;
  if (y >= a.g.ny || x >= a.g.nx) return;
  Gather<0, View> gat{{a.src, a.g}, a.r, 1.0 - a.r, a.shift, 0.0, 0.0};
  double f[9];
  gat(x, y, f);
  const Rates s{a.s3, a.snu, a.sq, a.s8};
  collide<FORCE, THIRD>(f, a.gx, a.gy, s);
  store9(a.dst, a.g, x, y, f);
}

// ---------------------------------------------------------------------------
// K1b: K periodic steps in one launch (temporal blocking).  A workgroup of
// 1024 threads owns a tile of 64 columns x (H - 2(K - 1)) rows.  The first
// step is computed for the tile and a (K - 1)-node halo
// around it (rows beyond a wall are skipped) and kept in LDS; each further
// step gathers from LDS for a region one node smaller on every side and
// overwrites LDS in place (barriers between reading and writing); the last
// writes the tile to HBM.  Per K steps a tile node costs
// (64 + 2(K - 1)) H / (64 (H - 2(K - 1))) x 72 B of reads and 72 B of writes
// instead of K x 144 B.  The gather and collision are K1's code, so K steps
// here equal K one-step launches bit for bit.
// ---------------------------------------------------------------------------
constexpr int kTileX = 64;   // tile columns
// Tiles are handed out in strips of kStripBands tile rows, each strip walked
// column by column: the tiles an XCD runs at the same time (consecutive
// logical blocks) then sit above and beside each other and share their halo
// rows and columns in that XCD's L2.  In row-major order the rows shared
// with the next band were read from HBM twice.
constexpr int kStripBands = 16;

// Populations of a tile region in LDS, [9][h][w], addressed with global
// (unwrapped) coordinates.
struct TileView {
  const double* P;
  int x0, y0;       // global coordinates of LDS column 0 and row 0
  int w, h;
  int nx_, ny_;
  __device__ __forceinline__ double at(int i, int x, int y) const {
    return P[(i * h + (y - y0)) * w + (x - x0)];
  }
  __device__ __forceinline__ int nx() const { return nx_; }
  __device__ __forceinline__ int ny() const { return ny_; }
};

// The HBM rows a multi-step tile reads and writes, addressed by 32-bit byte
// offsets from a workgroup-uniform base (row ybase, direction 0, lane 0):
// a load's address is one 32-bit sum of its row part, column part and
// direction slot added to a base in scalar registers, instead of a 64-bit
// index product per load.  Valid while the rows a tile touches
// (kTileRowsMax of them) span less than 4 GiB.
constexpr int kTileRowsMax = 17;   // H + 2 for the largest H

struct RowsView {
  const char* base;
  int ybase;
  uint32_t row_bytes;   // bytes per row of the device layout
  int lshift;
  int nx_, ny_;
  __device__ __forceinline__ uint32_t offset(int i, int x, int y) const {
    const uint32_t col = ((uint32_t)((x >> lshift) * 9 + i) << lshift) + (uint32_t)(x & ((1 << lshift) - 1));
    return (uint32_t)(y - ybase) * row_bytes + (col << 3);
  }
  __device__ __forceinline__ double at(int i, int x, int y) const {
    return *reinterpret_cast<const double*>(base + offset(i, x, y));
  }
  __device__ __forceinline__ int nx() const { return nx_; }
  __device__ __forceinline__ int ny() const { return ny_; }
};

// A whole population buffer of less than 4 GiB addressed by 32-bit byte
// offsets from its (uniform) base: the pressure kernels' HBM loads and
// stores, one 32-bit index per access instead of 64-bit products.
struct View32 {
  const char* base;
  Geo g;
  __device__ __forceinline__ uint32_t offset(int i, int x, int y) const {
    const uint32_t seg = (uint32_t)y * (uint32_t)g.nseg + (uint32_t)(x >> g.lshift);
    return (((seg * 9 + (uint32_t)i) << g.lshift) + (uint32_t)(x & ((1 << g.lshift) - 1))) << 3;
  }
  __device__ __forceinline__ const double* ptr(int i, int x, int y) const {
    return reinterpret_cast<const double*>(base + offset(i, x, y));
  }
  __device__ __forceinline__ double at(int i, int x, int y) const { return *ptr(i, x, y); }
  __device__ __forceinline__ int nx() const { return g.nx; }
  __device__ __forceinline__ int ny() const { return g.ny; }
};

template <int K>
constexpr int tile_w() {
  return kTileX + 2 * (K - 1);
}

// Threads of a multi-step workgroup: 16 wavefronts, enough for the first
// step's region ((64 + 2(K - 1)) x H <= 1024 nodes for the shipped H).
constexpr int kStepKThreads = 1024;

// Node of step k's region (k = 1 .. K: columns k - 1 .. W - k, rows
// k - 1 .. H - k of the LDS tile) taken by thread t.  The region's share of
// the tile's 64 columns comes first, one row per wavefront, so that every
// wavefront reads and writes whole aligned 512-byte row pieces of each
// direction slot and finds the same wall rule on all its lanes; the
// K - k halo columns on either side of those rows follow.  False for
// threads beyond the region.
template <int K, int H>
__device__ __forceinline__ bool region_node(int k, int t, int& lx, int& ly) {
  const int hw = K - k;
  const int rows = H - 2 * (k - 1);
  const int main = kTileX * rows;
  if (t < main) {
    lx = (K - 1) + (t & (kTileX - 1));
    ly = (k - 1) + t / kTileX;
    return true;
  }
  const int j = t - main;
  if (j >= 2 * hw * rows) return false;
  const int r = j / (2 * hw), c = j - r * 2 * hw;
  ly = (k - 1) + r;
  lx = c < hw ? (k - 1) + c : (K - 1) + kTileX + (c - hw);
  return true;
}

// Occupancy target: 8 waves per SIMD (at most 64 VGPRs; two to four steps
// need 54-58 with no spill), so two workgroups (and their 71-74 KB of LDS)
// share a CU.
template <bool FORCE, bool THIRD, int K, int H>
__global__ __launch_bounds__(kStepKThreads, 8) void k_stepk_periodic(StepArgs a) {
  constexpr int W = tile_w<K>();
  static_assert(W * H <= kStepKThreads, "first-step region larger than the workgroup");
  extern __shared__ double s1[];   // [9][H][W]
  const int nx = a.g.nx, ny = a.g.ny;
  const int ntx = (nx + kTileX - 1) / kTileX;
  const int nty = (ny + H - 2 * K + 1) / (H - 2 * (K - 1));
  const int b = logical_block(a.xcd_remap);
  const int strip = b / (ntx * kStripBands);
  const int rb = b - strip * (ntx * kStripBands);
  const int bands = min(kStripBands, nty - strip * kStripBands);   // the last strip may be shorter
  const int bx = rb / bands, by = strip * kStripBands + (rb - bx * bands);
  const int x0 = bx * kTileX - (K - 1), y0 = by * (H - 2 * (K - 1)) - (K - 1);   // LDS (0, 0)
  const int t = threadIdx.x;
  const Rates s{a.s3, a.snu, a.sq, a.s8};
  // the first row any step of this tile reads or writes
  const int ybase = y0 - 1 < 0 ? 0 : y0 - 1;
  const uint32_t row_bytes = (uint32_t)((a.g.nseg * 9) << a.g.lshift) << 3;
  const size_t base_off = (size_t)ybase * (size_t)((a.g.nseg * 9) << a.g.lshift);
  {
    int lx, ly;
    if (region_node<K, H>(1, t, lx, ly)) {
      const int x = x0 + lx, y = y0 + ly;
      if (y >= 0 && y < ny) {          // rows beyond a wall are skipped
        int xw = x % nx;               // x >= -(K - 1)
        if (xw < 0) xw += nx;
        const Gather<0, RowsView> gat{{reinterpret_cast<const char*>(a.src + base_off), ybase, row_bytes, a.g.lshift,
                                       nx, ny},
                                      a.r, 1.0 - a.r, a.shift, 0.0, 0.0};
        double f[9];
        gat(xw, y, f);
        collide<FORCE, THIRD>(f, a.gx, a.gy, s);
#pragma unroll
        for (int i = 0; i < 9; ++i) s1[(i * H + ly) * W + lx] = f[i];
      }
    }
  }
  const Gather<3, TileView> lds{{s1, x0, y0, W, H, nx, ny}, a.r, 1.0 - a.r, a.shift, 0.0, 0.0};
  // intermediate steps: gather and collide, barrier, overwrite in place
#pragma unroll
  for (int k = 2; k < K; ++k) {
    int lx, ly;
    bool in = region_node<K, H>(k, t, lx, ly);
    const int x = x0 + lx, y = y0 + ly;
    in = in && y >= 0 && y < ny;
    __syncthreads();
    double f[9];
    if (in) {
      lds(x, y, f);
      collide<FORCE, THIRD>(f, a.gx, a.gy, s);
    }
    __syncthreads();
    if (in) {
#pragma unroll
      for (int i = 0; i < 9; ++i) s1[(i * H + ly) * W + lx] = f[i];
    }
  }
  // last step: the tile itself, written to HBM
  __syncthreads();
  int lx, ly;
  if (region_node<K, H>(K, t, lx, ly)) {
    const int x = x0 + lx, y = y0 + ly;
    if (y >= 0 && y < ny && x < nx) {
      double f[9];
      lds(x, y, f);
      collide<FORCE, THIRD>(f, a.gx, a.gy, s);
      const RowsView out{reinterpret_cast<const char*>(a.dst + base_off), ybase, row_bytes, a.g.lshift, nx, ny};
      char* const q = reinterpret_cast<char*>(a.dst + base_off);
#pragma unroll
      for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(f[i], reinterpret_cast<double*>(q + out.offset(i, x, y)));
    }
  }
}

// ---------------------------------------------------------------------------
// K2: fused pressure-driven step.  Block = CX columns x ny rows (64 row
// lanes for taller channels), so that up to ny = 64 each thread owns one
// node and long narrow channels (2000 x 20: 250 workgroups) fill the chip.
// The centre-line density of each column (same step, pre-collision) sets
// the local Knudsen number Kn(x) = Kn_out rho_out / rho_c(x) (Section 3.2)
// and through Eqs. (18), (21) the column's s_nu and s_q.  With one node per thread the centre-row threads publish their own
// density through LDS; otherwise the first row lane gathers the centre rows.
// Workgroups take the XCD-aware order; interior ones gather with no
// x-boundary code, the first and last stage the two ghost columns in LDS
// (channels taller than 512 rows evaluate ghost populations inline).
// ---------------------------------------------------------------------------

// One workgroup's CX columns with the gather of MODE 3 (interior), 2 (ghost
// columns staged in s_ghost by this workgroup) or 1 (ghosts inline).
// s_rc: [2][CX] centre-row densities.  ONE: the workgroup is exactly ny rows
// tall (ny <= 64), one node per thread; otherwise it has 64 row lanes and
// each thread walks rows y, y + 64, ...  The two forms are separate kernel
// instances: the row loop needs about twice the registers, which would
// halve the waves in flight of the one-node form used by the paper's
// channels.  With staged ghosts every thread issues its own gather loads
// before the staging, so the two overlap; the few ghost-sourced values are
// patched in after the barrier.
template <int MODE, int CX, bool ONE>
__device__ __forceinline__ void pressure_columns(const StepArgs& a, const Gather<MODE, View>& gat, int blk, int nblk,
                                                 double (*s_rc)[CX], double* s_ghost) {
  const int tx = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
  const int x = blk * CX + tx;
  const int ny = a.g.ny, yc = ny / 2;
  const bool even = (ny & 1) == 0;
  auto stage = [&]() {
    if (MODE == 2) {
      fill_ghosts(gat.v, a.rho_in, a.rho_out, blk == 0, blk == nblk - 1, s_ghost, s_ghost + 9 * ny, ty * CX + tx,
                  CX * ry);
      __syncthreads();
    }
  };
  if constexpr (ONE) {
    const bool active = x < a.g.nx;
    double f[9];
    if constexpr (MODE == 2) {
      double A[9], B[4];
      if (active) gat.template load_sources<true>(x, ty, A, B);
      stage();
      if (active) {
        gat.patch_ghosts(x, ty, A, B);
        gat.combine(ty, A, B, f);
      }
    } else {
      if (active) gather_node(gat, x, ty, f);
    }
    if (active) {
      if (ty == yc) s_rc[0][tx] = sum9(f);
      if (even && ty == yc - 1) s_rc[1][tx] = sum9(f);
    }
    __syncthreads();
    if (!active) return;
    const double rc = even ? 0.5 * (s_rc[1][tx] + s_rc[0][tx]) : s_rc[0][tx];
    double snu, sq;
    local_rates(a.kn, a.rho_out, rc, a.c_tau, a.a, a.A2, a.tq_den, snu, sq);
    collide<false>(f, 0.0, 0.0, Rates{a.s3, snu, sq, a.s8});
    store9(a.dst, a.g, x, ty, f);
  } else {
    stage();
    if (ty < 2 && x < a.g.nx && (ty == 0 || even)) {
      double f[9];
      gather_node(gat, x, yc - ty, f);
      s_rc[ty][tx] = sum9(f);
    }
    __syncthreads();
    if (x >= a.g.nx) return;
    const double rc = even ? 0.5 * (s_rc[1][tx] + s_rc[0][tx]) : s_rc[0][tx];
    double snu, sq;
    local_rates(a.kn, a.rho_out, rc, a.c_tau, a.a, a.A2, a.tq_den, snu, sq);
    const Rates s{a.s3, snu, sq, a.s8};
    for (int y = ty; y < ny; y += ry) {
      double f[9];
      gather_node(gat, x, y, f);
      collide<false>(f, 0.0, 0.0, s);
      store9(a.dst, a.g, x, y, f);
    }
  }
}

// Column workgroup blk of nblk covering one channel (ONE: ny <= 64, so the
// ghost columns always fit in LDS).
template <int CX, bool ONE>
__device__ __forceinline__ void pressure_block(const StepArgs& a, int blk, int nblk, double (*s_rc)[CX],
                                               double* s_ghost) {
  const View v{a.src, a.g};
  const double omr = 1.0 - a.r;
  if (blk != 0 && blk != nblk - 1) {
    // every x - 1 and x + 1 of this workgroup lies inside the grid
    pressure_columns<3, CX, ONE>(a, Gather<3, View>{v, a.r, omr, a.shift, a.rho_in, a.rho_out}, blk, nblk, s_rc,
                                     nullptr);
  } else if (ONE || a.ghost_lds) {
    const int ny = a.g.ny;
    pressure_columns<2, CX, ONE>(
        a, Gather<2, View>{v, a.r, omr, a.shift, a.rho_in, a.rho_out, s_ghost, s_ghost + 9 * ny}, blk, nblk, s_rc,
        s_ghost);
  } else {
    pressure_columns<1, CX, ONE>(a, Gather<1, View>{v, a.r, omr, a.shift, a.rho_in, a.rho_out}, blk, nblk, s_rc,
                                     nullptr);
  }
}

// Threads of a column workgroup at most: CX * ny <= 1024 (ONE), CX * 64.
template <int CX, bool ONE>
constexpr int column_threads() {
  return ONE ? 1024 : CX * 64;
}

template <int CX, bool ONE>
__global__ __launch_bounds__((column_threads<CX, ONE>())) void k_step_pressure(StepArgs a) {
  extern __shared__ double s_ghost[];   // [2][9][ny] in the first / last workgroup
  __shared__ double s_rc[2][CX];
  pressure_block<CX, ONE>(a, logical_block(a.xcd_remap), (int)gridDim.x, s_rc, s_ghost);
}

// ---------------------------------------------------------------------------
// K2e: K = 2..4 pressure-driven steps in one launch, for channels of at most
// 48 rows.  A workgroup of (CX + 2(K - 1)) x ny threads owns CX columns; the
// first step is computed for them and K - 1 columns on each side (inlet /
// outlet ghost columns staged from HBM as in K2) and kept in LDS, each
// further step from LDS for a region one column narrower on each side, the
// last one stored to HBM.  A step whose region holds the first or last
// column of the channel rebuilds that ghost column from the previous step's
// LDS values, and every step takes its per-column rates from its own centre
// rows.  The gather, ghost, rate and collision arithmetic is K2's, so the
// result equals K launches of K2 bit for bit; a node update moves about
// ((CX + 2(K - 1)) / CX x 72 + 72) / K bytes of HBM traffic instead of 144.
// ---------------------------------------------------------------------------
template <int CX, int K>
constexpr int pressure_tile_w() {
  return CX + 2 * (K - 1);
}

// One step of a K2e workgroup: step k of K (LDS columns k - 1 .. W - k),
// gathered from HBM (the first step) or from LDS, kept in LDS or stored to
// HBM (the last).
template <int CX, int K>
__device__ __forceinline__ void pressurek_step(const StepArgs& a, int blk, double* lds,
                                               double (*s_rc)[pressure_tile_w<CX, K>()],
                                               double (*s_rate)[pressure_tile_w<CX, K>()], int k) {
  constexpr int W = pressure_tile_w<CX, K>();
  const int nx = a.g.nx, ny = a.g.ny;
  double* s1 = lds;                    // [9][ny][W]: the latest step kept
  double* gh = lds + 9 * ny * W;       // [2][9][ny]: ghost columns of the current step
  const int x0 = blk * CX - (K - 1);   // global column of LDS column 0
  int lx = threadIdx.x, ty = threadIdx.y;
  // Opaque copies per step: the compiler would otherwise compute the LDS
  // addresses of every step's gather up front and hold them (spilled to
  // scratch) across the steps.
  asm volatile("" : "+v"(lx), "+v"(ty));
  const int x = x0 + lx;
  const double omr = 1.0 - a.r;
  // step k covers global columns lo .. hi that exist
  const int lo = x0 + (k - 1), hi = x0 + W - k;
  const bool need_in = lo <= 0 && hi >= 0, need_out = lo <= nx - 1 && hi >= nx - 1;
  const bool valid = lx >= k - 1 && lx <= W - k && x >= 0 && x < nx;
  const TileView tv{s1, x0, 0, W, ny, nx, ny};
  if (need_in || need_out) {   // uniform across the workgroup
    const int tid = ty * W + lx, nthreads = W * ny;
    if (k == 1)
      fill_ghosts_lean(View32{reinterpret_cast<const char*>(a.src), a.g}, a.rho_in, a.rho_out, need_in, need_out, gh,
                       gh + 9 * ny, tid, nthreads);
    else
      fill_ghosts_lean(tv, a.rho_in, a.rho_out, need_in, need_out, gh, gh + 9 * ny, tid, nthreads);
    __syncthreads();
  }
  const int yc = ny / 2;
  const bool even = (ny & 1) == 0;
  double f[9];
  if (valid) {
    if (k == 1) {
      const View32 v{reinterpret_cast<const char*>(a.src), a.g};
      if (need_in || need_out)
        Gather<2, View32>{v, a.r, omr, a.shift, a.rho_in, a.rho_out, gh, gh + 9 * ny}(x, ty, f);
      else
        Gather<3, View32>{v, a.r, omr, a.shift, a.rho_in, a.rho_out}(x, ty, f);
    } else {
      if (need_in || need_out)
        Gather<2, TileView>{tv, a.r, omr, a.shift, a.rho_in, a.rho_out, gh, gh + 9 * ny}(x, ty, f);
      else
        Gather<3, TileView>{tv, a.r, omr, a.shift, a.rho_in, a.rho_out}(x, ty, f);
    }
    if (ty == yc) s_rc[0][lx] = sum9(f);
    if (even && ty == yc - 1) s_rc[1][lx] = sum9(f);
  }
  __syncthreads();   // centre densities published; every read of step k - 1 done
  // the column's rates, once per column (the same arithmetic as every node
  // of the column evaluating them)
  if (valid && ty == 0) {
    const double rc = even ? 0.5 * (s_rc[1][lx] + s_rc[0][lx]) : s_rc[0][lx];
    local_rates(a.kn, a.rho_out, rc, a.c_tau, a.a, a.A2, a.tq_den, s_rate[0][lx], s_rate[1][lx]);
  }
  __syncthreads();
  if (valid) {
    collide<false>(f, 0.0, 0.0, Rates{a.s3, s_rate[0][lx], s_rate[1][lx], a.s8});
    if (k < K) {
#pragma unroll
      for (int i = 0; i < 9; ++i) s1[(i * ny + ty) * W + lx] = f[i];
    } else {
      const View32 out{reinterpret_cast<const char*>(a.dst), a.g};
      char* const q = reinterpret_cast<char*>(a.dst);
#pragma unroll
      for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(f[i], reinterpret_cast<double*>(q + out.offset(i, x, ty)));
    }
  }
}

// s_rc: [2][W] centre-row densities, s_rate: [2][W] the columns' s_nu, s_q.
template <int CX, int K>
__device__ __forceinline__ void pressurek_block(const StepArgs& a, int blk, double* lds,
                                                double (*s_rc)[pressure_tile_w<CX, K>()],
                                                double (*s_rate)[pressure_tile_w<CX, K>()]) {
  pressurek_step<CX, K>(a, blk, lds, s_rc, s_rate, 1);
#pragma unroll
  for (int k = 2; k <= K; ++k) {
    __syncthreads();   // step k - 1 is in LDS
    pressurek_step<CX, K>(a, blk, lds, s_rc, s_rate, k);
  }
}

template <int CX, int K>
__global__ __launch_bounds__(1024) void k_stepk_pressure(StepArgs a) {
  extern __shared__ double lds[];   // [9][ny][W] + [2][9][ny]
  __shared__ double s_rc[2][pressure_tile_w<CX, K>()], s_rate[2][pressure_tile_w<CX, K>()];
  pressurek_block<CX, K>(a, logical_block(a.xcd_remap), lds, s_rc, s_rate);
}

// ---------------------------------------------------------------------------
// K2c: one step of a batch of pressure-driven channels of the same grid
// (the mass-flow sweep of Section 3.2), in one launch: workgroup b serves
// column block b % nblk of channel live[b / nblk] with that channel's
// parameters, the same arithmetic as K2 (bitwise the same populations).
// The launch covers the channels still running (the host keeps the list);
// a channel found stopped is skipped.
// ---------------------------------------------------------------------------
// Step arguments of channel c of a batch.
__device__ __forceinline__ StepArgs channel_args(const PBatchArgs& p, int c) {
  const PChan ch = p.ch[c];
  StepArgs a{};
  a.src = p.buf[p.par] + (size_t)c * p.stride;
  a.dst = p.buf[p.par ^ 1] + (size_t)c * p.stride;
  a.g = p.g;
  a.mode = 1;
  a.shift = p.shift;
  a.ghost_lds = p.ghost_lds;
  a.r = ch.r;
  a.s3 = ch.s3;
  a.s8 = ch.s8;
  a.kn = ch.kn;
  a.a = ch.a;
  a.A2 = ch.A2;
  a.tq_den = ch.tq_den;
  a.c_tau = p.c_tau;
  a.rho_in = ch.rho_in;
  a.rho_out = ch.rho_out;
  if (p.col_rates) {
    a.col_rates = p.col_rates + (size_t)c * 2 * p.g.nx;
    a.ghosts = p.ghosts + (size_t)c * 18 * p.g.ny;
  }
  return a;
}

template <int CX, bool ONE>
__global__ __launch_bounds__((column_threads<CX, ONE>())) void k_pbatch_step(PBatchArgs p) {
  extern __shared__ double s_ghost[];
  __shared__ double s_rc[2][CX];
  const int b = logical_block(p.xcd_remap);
  const int k = b / p.nblk;
  const int c = p.live[k];
  if (!p.state[c].active) return;
  pressure_block<CX, ONE>(channel_args(p, c), b - k * p.nblk, p.nblk, s_rc, s_ghost);
}

// K steps of every running channel in one launch (K2e per channel).
template <int CX, int K>
__global__ __launch_bounds__(1024) void k_pbatch_stepk(PBatchArgs p) {
  extern __shared__ double lds[];
  __shared__ double s_rc[2][pressure_tile_w<CX, K>()], s_rate[2][pressure_tile_w<CX, K>()];
  const int b = logical_block(p.xcd_remap);
  const int k = b / p.nblk;
  const int c = p.live[k];
  if (!p.state[c].active) return;
  pressurek_block<CX, K>(channel_args(p, c), b - k * p.nblk, lds, s_rc, s_rate);
}

// ---------------------------------------------------------------------------
// K2b: pressure-driven step for large grids, in two launches.  The prep
// kernel takes each column's centre-line density from the same step's
// gather, turns it into the column's s_nu, s_q (same arithmetic as K2), and
// builds the two ghost columns; the row kernel then streams the grid in the
// periodic kernel's order (one thread per node, whole row segments per
// workgroup), reading the rates and ghosts from those arrays.  Bitwise the
// same result as K2.
// ---------------------------------------------------------------------------
// Prep work item `bid` of a channel: blocks below ncb compute the rates of
// 256 columns each, the rest build 256 ghost rows each.
__device__ __forceinline__ void pressure_prep_block(const StepArgs& a, int bid, int ncb) {
  const int nx = a.g.nx, ny = a.g.ny;
  const View v{a.src, a.g};
  if (bid < ncb) {
    const int x = bid * 256 + threadIdx.x;
    if (x >= nx) return;
    const Gather<1, View> gat{v, a.r, 1.0 - a.r, a.shift, a.rho_in, a.rho_out};
    const int yc = ny / 2;
    double f[9];
    gather_node(gat, x, yc, f);
    double rc = sum9(f);
    if ((ny & 1) == 0) {
      gather_node(gat, x, yc - 1, f);
      rc = 0.5 * (sum9(f) + rc);
    }
    double snu, sq;
    local_rates(a.kn, a.rho_out, rc, a.c_tau, a.a, a.A2, a.tq_den, snu, sq);
    a.col_rates[x] = snu;
    a.col_rates[nx + x] = sq;
  } else {
    // ghost rows: j < ny inlet row j, else outlet row j - ny
    const int j = (bid - ncb) * 256 + threadIdx.x;
    if (j >= 2 * ny) return;
    const bool inlet = j < ny;
    const int y = inlet ? j : j - ny;
    double g[9];
    ghost_row(v, inlet, y, inlet ? a.rho_in : a.rho_out, g);
#pragma unroll
    for (int i = 0; i < 9; ++i) a.ghosts[(inlet ? 0 : 9 * ny) + i * ny + y] = g[i];
  }
}

// Row-kernel node update of padded node t (device-layout order).
__device__ __forceinline__ void pressure_rows_node(const StepArgs& a, size_t t) {
  const int lane = (int)(t & (((size_t)1 << a.g.lshift) - 1));
  const size_t rest = t >> a.g.lshift;
  const int y = (int)(rest / (size_t)a.g.nseg);
  const int x = (int)(rest - (size_t)y * a.g.nseg) * (1 << a.g.lshift) + lane;
  if (y >= a.g.ny || x >= a.g.nx) return;
  const int ny = a.g.ny;
  const Gather<2, View> gat{{a.src, a.g}, a.r, 1.0 - a.r, a.shift, a.rho_in, a.rho_out, a.ghosts,
                            a.ghosts + 9 * ny};
  // a wave covers consecutive x of one row: the wall branches do not diverge
  double f[9];
  gat(x, y, f);
  collide<false>(f, 0.0, 0.0, Rates{a.s3, a.col_rates[x], a.col_rates[a.g.nx + x], a.s8});
  store9(a.dst, a.g, x, y, f);
}

__global__ __launch_bounds__(256) void k_pressure_prep(StepArgs a) {
  pressure_prep_block(a, blockIdx.x, (a.g.nx + 255) / 256);
}

__global__ __launch_bounds__(1024) void k_step_pressure_rows(StepArgs a) {
  pressure_rows_node(a, (size_t)logical_block(a.xcd_remap) * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// K2d: row-kernel form of K2c for batches of many channels: per step a prep
// launch over every running channel, then one row-streaming launch over
// all of them (channel-major, each channel's grid in device-layout order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pbatch_prep(PBatchArgs p) {
  const int ncb = (p.g.nx + 255) / 256;
  const int per = ncb + (2 * p.g.ny + 255) / 256;
  const int k = blockIdx.x / per;
  const int c = p.live[k];
  if (!p.state[c].active) return;
  pressure_prep_block(channel_args(p, c), (int)blockIdx.x - k * per, ncb);
}

__global__ __launch_bounds__(1024) void k_pbatch_rows(PBatchArgs p) {
  const int b = logical_block(p.xcd_remap);
  const int k = b / p.nblk;
  const int c = p.live[k];
  if (!p.state[c].active) return;
  pressure_rows_node(channel_args(p, c), (size_t)(b - k * p.nblk) * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// K3: initial state (logical node order; node = y * nx + x).
// ---------------------------------------------------------------------------
__global__ void k_init(InitArgs a) {
  const size_t n = (size_t)a.g.nx * (size_t)a.g.ny;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(idx / (size_t)a.g.nx);
    const int x = (int)(idx - (size_t)y * a.g.nx);
    double rho = a.rho0, ux = a.ux0, uy = a.uy0;
    if (a.kind == 1) {
      const double xc = (double)x + 0.5;
      rho = a.rho_in - (a.rho_in - a.rho_out) * xc / (double)a.g.nx;
      ux = 0.0;
      uy = 0.0;
    }
    double e[9];
    equilibrium(rho, ux, uy, e);
    if (a.kind == 2) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const uint64_t key = a.seed ^ (9ull * (uint64_t)idx + (uint64_t)i);
        const double U = (double)(splitmix64_first(key) >> 11) * (1.0 / 9007199254740992.0);
        e[i] += a.amp * (2.0 * U - 1.0);
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) a.dst[a.g.index(i, x, y)] = e[i];
  }
}

// ABI layout [9][ny][nx] <-> device layout.
template <bool EXPORT>
__global__ void k_convert(const double* __restrict__ src, Geo g, double* __restrict__ dst) {
  const size_t plane = (size_t)g.nx * (size_t)g.ny;
  const size_t n = 9 * plane;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(k / plane);
    const size_t node = k - (size_t)i * plane;
    const int y = (int)(node / (size_t)g.nx);
    const int x = (int)(node - (size_t)y * g.nx);
    if (EXPORT)
      dst[k] = src[g.index(i, x, y)];
    else
      dst[g.index(i, x, y)] = src[k];
  }
}

// ---------------------------------------------------------------------------
// K4: diagnostics of the pre-collision state.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void k_moments(DiagArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= a.g.nx) return;
  Gather<MODE, View> gat{{a.src, a.g}, a.r, 1.0 - a.r, a.shift, a.rho_in, a.rho_out};
  double f[9];
  gather_node(gat, x, y, f);
  double rho, ux, uy;
  rho_u(f, rho, ux, uy);
  ux += 0.5 * a.gx;
  uy += 0.5 * a.gy;
  const size_t idx = (size_t)y * a.g.nx + x;
  if (a.rho) a.rho[idx] = rho;
  if (a.ux) a.ux[idx] = ux;
  if (a.uy) a.uy[idx] = uy;
}

// Per-column sums.  A workgroup owns kColLanes adjacent columns, one per
// lane, so every population load of a wavefront is one contiguous 512-byte
// row piece; its kColWaves wavefronts split the rows (wave w takes rows w,
// w + kColWaves, ...), and the per-wave partial sums of each column are
// added in wave order through LDS: a fixed summation order.
constexpr int kColLanes = 64;
constexpr int kColWaves = 16;

template <int MODE, class V>
__global__ __launch_bounds__(kColLanes * kColWaves) void k_column_sums(DiagArgs a, V v) {
  __shared__ double sm[kColWaves][kColLanes], su[kColWaves][kColLanes];
  const int lane = threadIdx.x & (kColLanes - 1), w = threadIdx.x / kColLanes;
  const int x = blockIdx.x * kColLanes + lane;
  const int nx = v.nx(), ny = v.ny();
  Gather<MODE, V> gat{v, a.r, 1.0 - a.r, a.shift, a.rho_in, a.rho_out};
  double accm = 0.0, accu = 0.0;
  if (x < nx) {
    for (int y = w; y < ny; y += kColWaves) {
      double f[9];
      gather_node(gat, x, y, f);
      double rho, ux, uy;
      rho_u(f, rho, ux, uy);
      ux += 0.5 * a.gx;
      accm += rho * ux;
      accu += ux;
    }
  }
  sm[w][lane] = accm;
  su[w][lane] = accu;
  __syncthreads();
  if (w == 0 && x < nx) {
    double m = sm[0][lane], u = su[0][lane];
#pragma unroll
    for (int k = 1; k < kColWaves; ++k) {
      m += sm[k][lane];
      u += su[k][lane];
    }
    double f[9];
    const int yc = ny / 2;
    gather_node(gat, x, yc, f);
    double rc = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    if ((ny & 1) == 0) {
      gather_node(gat, x, yc - 1, f);
      rc = 0.5 * ((f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]) + rc);
    }
    if (a.m) a.m[x] = m;
    if (a.su) a.su[x] = u;
    if (a.rhoc) a.rhoc[x] = rc;
  }
}

// Sum of n values in a fixed order (one workgroup of 256 threads): strided
// per-thread sums, a wavefront butterfly, then the four wavefront totals in
// order; divided by `divisor` (n for a mean, 1 for a plain sum).
__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ v, int n, double divisor,
                                             double* __restrict__ out) {
  __shared__ double s[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = ((s[0] + s[1]) + (s[2] + s[3])) / divisor;
}

// delta p(x) = (rho_c/3 - p_l(x)) / p_out, p_l linear from p_in to p_out.
__global__ void k_pressure_dev(const double* __restrict__ rhoc, int nx, double rho_in, double rho_out,
                               double* __restrict__ dp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const double p_out = rho_out / 3.0, p_in = rho_in / 3.0;
  const double pl = p_in - (p_in - p_out) * ((double)x + 0.5) / (double)nx;
  dp[x] = (rhoc[x] / 3.0 - pl) / p_out;
}

// Non-finite count over the logical nodes: per-block partials, then one
// block sums them in order.
__global__ __launch_bounds__(256) void k_nonfinite_partial(const double* __restrict__ p, Geo g,
                                                           double* __restrict__ partial) {
  __shared__ double s[4];
  const size_t n = (size_t)g.nx * (size_t)g.ny;
  double cnt = 0.0;
  for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
    const int y = (int)(k / (size_t)g.nx);
    const int x = (int)(k - (size_t)y * g.nx);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double v = p[g.index(i, x, y)];
      cnt += (v - v == 0.0) ? 0.0 : 1.0;   // inf - inf and NaN - NaN are NaN
    }
  }
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

unsigned grid_for(size_t n, unsigned cap = 65536) {
  size_t b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b == 0) b = 1;
  return (unsigned)b;
}

// Shape of the column kernels: CX adjacent columns x ry rows, ry = ny for
// ny <= 64 (one node per thread, no idle rows) else 64.  CX is the widest of
// 64, 32, 16, 8, 4 with CX * ry <= 1024 that still leaves about one
// workgroup per CU over all nch channels (longer coalesced row pieces per
// wave), else the narrowest.  Measured on one channel: 4000 x 40 10.2 ->
// 6.3 us per step against 256-thread workgroups; 2000 x 20 keeps 8 columns.
struct ColumnShape {
  int cx, ry, nblk;   // nblk: column workgroups per channel
  bool one;           // ny <= 64: one node per thread
};

ColumnShape column_shape(const Geo& g, int nch, int cus) {
  ColumnShape s;
  s.one = g.ny <= 64;
  s.ry = s.one ? g.ny : 64;
  const long enough = cus > 0 ? cus - cus / 10 : 230;
  for (const int cand : {64, 32, 16, 8, 4}) {
    if (cand * s.ry > (s.one ? 1024 : 512)) continue;
    s.cx = cand;   // the narrowest one if none leaves enough workgroups
    if ((long)nch * ((g.nx + cand - 1) / cand) >= enough) break;
  }
  s.nblk = (g.nx + s.cx - 1) / s.cx;
  return s;
}

size_t ghost_lds_bytes(const Geo& g) {
  return g.ny <= kGhostLdsMaxNy ? 2 * 9 * (size_t)g.ny * sizeof(double) : 0;
}

// Launch LAUNCH(CX, ONE) for the template instance that shape s names.
#define CLB_COLUMN_DISPATCH(s, LAUNCH)         \
  do {                                         \
    if (!(s).one) {                            \
      if ((s).cx == 8) LAUNCH(8, false);       \
      else LAUNCH(4, false);                   \
    } else {                                   \
      if ((s).cx == 64) LAUNCH(64, true);      \
      else if ((s).cx == 32) LAUNCH(32, true); \
      else if ((s).cx == 16) LAUNCH(16, true); \
      else if ((s).cx == 8) LAUNCH(8, true);   \
      else LAUNCH(4, true);                    \
    }                                          \
  } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
// LDS reserved (never touched) by each periodic step workgroup so that at
// most kStepThreadsPerCU threads share a CU.  The periodic step needs few
// registers and would otherwise run 32 waves per CU; measured on the
// 32768 x 2048 step, 16 waves per CU (one 1024-thread workgroup) stream about
// 4% faster.  Returns 0 (no cap) when the device does not allow the size.
hipError_t periodic_step_lds(int block_x, size_t* bytes) {
  *bytes = 0;
  int dev = 0, lds_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  if (e != hipSuccess) return e;
  const int per_cu = kStepThreadsPerCU / block_x > 1 ? kStepThreadsPerCU / block_x : 1;
  const size_t want = (size_t)lds_cu / (size_t)(per_cu + 1) + 256;   // per_cu + 1 workgroups no longer fit
  if (want * (size_t)per_cu > (size_t)lds_cu) return hipSuccess;
  if (hipFuncSetAttribute((const void*)k_step_periodic<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)want) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_step_periodic<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)want) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_step_periodic<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)want) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_step_pressure_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)want) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_pbatch_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) !=
          hipSuccess) {
    (void)hipGetLastError();
    return hipSuccess;
  }
  *bytes = want;
  return hipSuccess;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

hipError_t launch_step(const StepArgs& a, int block_x, hipStream_t st, size_t lds_reserve) {
  if (a.mode == 0) {
    const size_t threads = a.g.padded_nodes();
    const dim3 grid((unsigned)((threads + block_x - 1) / block_x));
    if ((a.gx != 0.0 || a.gy != 0.0) && a.forcing)
      k_step_periodic<true, true><<<grid, block_x, lds_reserve, st>>>(a);
    else if (a.gx != 0.0 || a.gy != 0.0)
      k_step_periodic<true, false><<<grid, block_x, lds_reserve, st>>>(a);
    else
      k_step_periodic<false, false><<<grid, block_x, lds_reserve, st>>>(a);
  } else if (a.col_rates && a.ghosts &&
             (a.pressure_path == 2 || (a.pressure_path == 0 && (size_t)a.g.nx * a.g.ny >= kPressureRowNodes))) {
    k_pressure_prep<<<(a.g.nx + 255) / 256 + (2 * a.g.ny + 255) / 256, 256, 0, st>>>(a);
    const size_t threads = a.g.padded_nodes();
    const dim3 grid((unsigned)((threads + block_x - 1) / block_x));
    k_step_pressure_rows<<<grid, block_x, lds_reserve, st>>>(a);
  } else {
    StepArgs b = a;
    b.ghost_lds = a.g.ny <= kGhostLdsMaxNy ? 1 : 0;
    const ColumnShape s = column_shape(a.g, 1, a.cus);
    const dim3 pgrid((unsigned)s.nblk);
#define CLB_PRESSURE_LAUNCH(CXV, ONEV) \
  k_step_pressure<CXV, ONEV><<<pgrid, dim3(CXV, s.ry), ghost_lds_bytes(a.g), st>>>(b)
    CLB_COLUMN_DISPATCH(s, CLB_PRESSURE_LAUNCH);
#undef CLB_PRESSURE_LAUNCH
  }
  return hipGetLastError();
}

// Multi-step pressure launches: channels of at most kPressureMultiStepRows rows
// on the column kernel's path (grids that take the row kernel step one at a
// time).  Measured with two steps per launch, us per step one / two: 2000 x
// 20 4.35 / 3.48, 4000 x 40 6.37 / 4.99, 8192 x 40 11.75 / 8.74, 32768 x 16
// 15.45 / 14.65, but 16384 x 64 33.0 / 34.1 (8-column tiles: the halo
// columns cost more than the second launch saves).  With the column rates
// evaluated once per column, 4000 x 40 takes 4.68 / 4.48 / 4.14 us per step
// at two / three / four steps per launch (16-column tiles; 8-column tiles
// 5.04 / 4.75 / 6.07), the batch of 16 channels of 2000 x 20 15.4 / 13.9 /
// 12.4 us (32-column tiles).
constexpr int kPressureMultiStepRows = 48;

// (The multi-step kernels address a buffer by 32-bit byte offsets.)
bool buffer_below_4gib(const Geo& g) { return g.size() * sizeof(double) <= 0xFFFFFFFFull; }

bool pressure_multi_step_ok(const StepArgs& a) {
  const bool rows = a.col_rates && a.ghosts &&
                    (a.pressure_path == 2 || (a.pressure_path == 0 && (size_t)a.g.nx * a.g.ny >= kPressureRowNodes));
  return a.mode == 1 && a.g.ny <= kPressureMultiStepRows && !rows && buffer_below_4gib(a.g);
}

// Width of K2e: the widest of 32, 16, 8 columns with (CX + 2(k - 1)) ny <=
// 1024 that leaves about one workgroup per CU over nch channels, else 8
// (which fits every k <= 4 up to 48 rows).
int stepk_pressure_cx(const Geo& g, int nch, int cus, int k) {
  const long enough = cus > 0 ? cus - cus / 10 : 230;
  for (const int cand : {32, 16}) {
    if ((cand + 2 * (k - 1)) * g.ny > 1024) continue;
    if ((long)nch * ((g.nx + cand - 1) / cand) >= enough) return cand;
  }
  return 8;
}

// [9][ny][W] populations and [2][9][ny] ghost columns.
size_t stepk_pressure_lds(const Geo& g, int cx, int k) {
  return (9 * (size_t)g.ny * (cx + 2 * (k - 1)) + 18 * (size_t)g.ny) * sizeof(double);
}

// LDS of a K2e workgroup at most: (CX + 2(k - 1)) ny <= 1024 nodes of 9
// doubles plus two ghost columns of at most 48 rows.
constexpr int kStepKPressureLdsMax = (9 * 1024 + 18 * kPressureMultiStepRows) * (int)sizeof(double);

template <int CX, int K>
hipError_t pressure_allow() {
  for (const void* f : {(const void*)k_stepk_pressure<CX, K>, (const void*)k_pbatch_stepk<CX, K>}) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kStepKPressureLdsMax);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Launch LAUNCH(CX, K) for the K2e instance of width cx and k steps.
#define CLB_STEPK_PRESSURE_DISPATCH(cx, k, LAUNCH) \
  do {                                             \
    if ((cx) == 32) {                              \
      if ((k) == 4) LAUNCH(32, 4);                 \
      else if ((k) == 3) LAUNCH(32, 3);            \
      else LAUNCH(32, 2);                          \
    } else if ((cx) == 16) {                       \
      if ((k) == 4) LAUNCH(16, 4);                 \
      else if ((k) == 3) LAUNCH(16, 3);            \
      else LAUNCH(16, 2);                          \
    } else {                                       \
      if ((k) == 4) LAUNCH(8, 4);                  \
      else if ((k) == 3) LAUNCH(8, 3);             \
      else LAUNCH(8, 2);                           \
    }                                              \
  } while (0)

hipError_t launch_stepk_pressure(const StepArgs& a, int k, hipStream_t st) {
  const int ny = a.g.ny;
  const int cx = stepk_pressure_cx(a.g, 1, a.cus, k);
  const dim3 grid((unsigned)((a.g.nx + cx - 1) / cx)), block(cx + 2 * (k - 1), ny);
  const size_t lds = stepk_pressure_lds(a.g, cx, k);
#define CLB_LAUNCH(CXV, KV) k_stepk_pressure<CXV, KV><<<grid, block, lds, st>>>(a)
  CLB_STEPK_PRESSURE_DISPATCH(cx, k, CLB_LAUNCH);
#undef CLB_LAUNCH
  return hipGetLastError();
}

bool pbatch_multi_step_ok(const PBatchArgs& a) {
  const bool rows = a.col_rates && a.ghosts &&
                    (a.path == 2 || (a.path == 0 && (size_t)a.nch * a.g.nx * a.g.ny >= kPBatchRowNodes));
  return a.g.ny <= kPressureMultiStepRows && !rows && buffer_below_4gib(a.g);
}

hipError_t launch_pbatch_stepk(const PBatchArgs& a, int k, hipStream_t st) {
  const int ny = a.g.ny;
  const int cx = stepk_pressure_cx(a.g, a.nch, a.cus, k);
  PBatchArgs b = a;
  b.nblk = (a.g.nx + cx - 1) / cx;
  const dim3 grid((unsigned)((size_t)b.nblk * a.nch)), block(cx + 2 * (k - 1), ny);
  const size_t lds = stepk_pressure_lds(a.g, cx, k);
#define CLB_LAUNCH(CXV, KV) k_pbatch_stepk<CXV, KV><<<grid, block, lds, st>>>(b)
  CLB_STEPK_PRESSURE_DISPATCH(cx, k, CLB_LAUNCH);
#undef CLB_LAUNCH
  return hipGetLastError();
}

hipError_t launch_pbatch_step(const PBatchArgs& a, hipStream_t st, size_t lds_reserve) {
  if (a.col_rates && a.ghosts &&
      (a.path == 2 || (a.path == 0 && (size_t)a.nch * a.g.nx * a.g.ny >= kPBatchRowNodes))) {
    PBatchArgs b = a;
    const int per = (a.g.nx + 255) / 256 + (2 * a.g.ny + 255) / 256;
    k_pbatch_prep<<<(unsigned)((size_t)per * a.nch), 256, 0, st>>>(b);
    b.nblk = (int)((a.g.padded_nodes() + 1023) / 1024);
    k_pbatch_rows<<<(unsigned)((size_t)b.nblk * a.nch), 1024, lds_reserve, st>>>(b);
    return hipGetLastError();
  }
  const ColumnShape s = column_shape(a.g, a.nch, a.cus);
  PBatchArgs b = a;
  b.ghost_lds = a.g.ny <= kGhostLdsMaxNy ? 1 : 0;
  b.nblk = s.nblk;
  const dim3 grid((unsigned)((size_t)s.nblk * a.nch));
#define CLB_PBATCH_LAUNCH(CXV, ONEV) \
  k_pbatch_step<CXV, ONEV><<<grid, dim3(CXV, s.ry), ghost_lds_bytes(a.g), st>>>(b)
  CLB_COLUMN_DISPATCH(s, CLB_PBATCH_LAUNCH);
#undef CLB_PBATCH_LAUNCH
  return hipGetLastError();
}

// Rows per tile of K1b for K = 2, 3, 4 steps per launch (at most 1024
// threads: 66 x 15, 68 x 15, 70 x 14).
template <int K>
constexpr int stepk_h() {
  return K == 2 ? 15 : (K == 3 ? 15 : 14);
}

template <int K>
size_t stepk_lds() {
  return 9 * (size_t)stepk_h<K>() * tile_w<K>() * sizeof(double);
}

template <int K>
hipError_t stepk_allow() {
  constexpr int H = stepk_h<K>();
  const int bytes = (int)stepk_lds<K>();
  for (const void* k : {(const void*)k_stepk_periodic<true, true, K, H>,
                        (const void*)k_stepk_periodic<true, false, K, H>,
                        (const void*)k_stepk_periodic<false, false, K, H>}) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int K>
hipError_t launch_stepk_t(const StepArgs& a, hipStream_t st) {
  constexpr int H = stepk_h<K>();
  const size_t tiles =
      (size_t)((a.g.nx + kTileX - 1) / kTileX) * (size_t)((a.g.ny + H - 2 * K + 1) / (H - 2 * (K - 1)));
  const dim3 grid((unsigned)tiles), block(kStepKThreads);
  const size_t lds = stepk_lds<K>();
  if ((a.gx != 0.0 || a.gy != 0.0) && a.forcing)
    k_stepk_periodic<true, true, K, H><<<grid, block, lds, st>>>(a);
  else if (a.gx != 0.0 || a.gy != 0.0)
    k_stepk_periodic<true, false, K, H><<<grid, block, lds, st>>>(a);
  else
    k_stepk_periodic<false, false, K, H><<<grid, block, lds, st>>>(a);
  return hipGetLastError();
}

// Several periodic steps per launch pay only on grids at least one tile
// wide: around a narrower channel (the 4-column channels of the Kn sweep)
// the 64-column tile recomputes the few real columns many times over (a
// loop of 64 such single-channel runs took 3.6 s instead of 2.7 s).
// The tiles also address their rows with 32-bit offsets (RowsView): rows of
// more than 4 GiB / kTileRowsMax (channels of more than 3.5 M columns) take
// one step per launch.
bool periodic_multi_step_ok(const StepArgs& a) {
  const size_t row_bytes = ((size_t)a.g.nseg * 9 << a.g.lshift) * sizeof(double);
  return a.mode == 0 && a.g.nx >= kTileX && (size_t)kTileRowsMax * row_bytes <= 0xFFFFFFFFull;
}

hipError_t stepk_setup() {
  hipError_t e = stepk_allow<2>();
  if (e == hipSuccess) e = stepk_allow<3>();
  if (e == hipSuccess) e = stepk_allow<4>();
  if (e == hipSuccess) e = pressure_allow<32, 2>();
  if (e == hipSuccess) e = pressure_allow<32, 3>();
  if (e == hipSuccess) e = pressure_allow<32, 4>();
  if (e == hipSuccess) e = pressure_allow<16, 2>();
  if (e == hipSuccess) e = pressure_allow<16, 3>();
  if (e == hipSuccess) e = pressure_allow<16, 4>();
  if (e == hipSuccess) e = pressure_allow<8, 2>();
  if (e == hipSuccess) e = pressure_allow<8, 3>();
  if (e == hipSuccess) e = pressure_allow<8, 4>();
  return e;
}

hipError_t launch_stepk(const StepArgs& a, int k, hipStream_t st) {
  if (k == 4) return launch_stepk_t<4>(a, st);
  if (k == 3) return launch_stepk_t<3>(a, st);
  return launch_stepk_t<2>(a, st);
}

namespace {
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Non-temporal loads and stores: the copied data is touched once, and the
// streaming hint keeps it from displacing the last-level cache (6.5 TB/s
// on MI355X against 6.25 with ordinary accesses).
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}
}  // namespace

hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  const size_t blocks = (n16 + 255) / 256;
  k_copy16<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(static_cast<const u32x4*>(src), static_cast<u32x4*>(dst),
                                                          n16);
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t st) {
  k_init<<<grid_for((size_t)a.g.nx * a.g.ny), 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_export(const double* src, const Geo& g, double* out, hipStream_t st) {
  k_convert<true><<<grid_for(9 * (size_t)g.nx * g.ny), 256, 0, st>>>(src, g, out);
  return hipGetLastError();
}

hipError_t launch_import(const double* in, const Geo& g, double* dst, hipStream_t st) {
  k_convert<false><<<grid_for(9 * (size_t)g.nx * g.ny), 256, 0, st>>>(in, g, dst);
  return hipGetLastError();
}

hipError_t launch_moments(const DiagArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.g.nx + 255) / 256), (unsigned)a.g.ny);
  if (a.mode == 0)
    k_moments<0><<<grid, 256, 0, st>>>(a);
  else
    k_moments<1><<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

template <class V>
hipError_t launch_column_sums_v(const DiagArgs& a, const V& v, hipStream_t st) {
  const dim3 grid((unsigned)((a.g.nx + kColLanes - 1) / kColLanes));
  if (a.mode == 0)
    k_column_sums<0, V><<<grid, kColLanes * kColWaves, 0, st>>>(a, v);
  else
    k_column_sums<1, V><<<grid, kColLanes * kColWaves, 0, st>>>(a, v);
  return hipGetLastError();
}

hipError_t launch_column_sums(const DiagArgs& a, hipStream_t st) {
  return launch_column_sums_v(a, View{a.src, a.g}, st);
}

hipError_t launch_column_sums_plane(const DiagArgs& a, const double* P, hipStream_t st) {
  return launch_column_sums_v(a, PlaneView{P, a.g.nx, a.g.ny}, st);
}

hipError_t launch_mean(const double* v, int n, double* out, hipStream_t st) {
  k_sum<<<1, 256, 0, st>>>(v, n, (double)n, out);
  return hipGetLastError();
}

hipError_t launch_pressure_dev(const double* rhoc, int nx, double rho_in, double rho_out, double* dp,
                               hipStream_t st) {
  k_pressure_dev<<<(nx + 255) / 256, 256, 0, st>>>(rhoc, nx, rho_in, rho_out, dp);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double* p, const Geo& g, double* partial, int nblocks, double* out,
                            hipStream_t st) {
  k_nonfinite_partial<<<nblocks, 256, 0, st>>>(p, g, partial);
  k_sum<<<1, 256, 0, st>>>(partial, nblocks, 1.0, out);
  return hipGetLastError();
}

}  // namespace clb
