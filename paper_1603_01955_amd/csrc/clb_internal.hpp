// Internal declarations shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace clb {

// Device layout of one population buffer: array of structures of arrays,
// [y][segment][i][lane] with L = 2^lshift lanes per row segment.  Each row
// segment keeps its nine directions in one contiguous 72*L-byte block, so a
// block of threads streams through few DRAM pages; x = segment * L + lane,
// lanes >= nx in the last segment are padding and never read.
struct Geo {
  int nx, ny;
  int lshift;   // log2 L
  int nseg;     // segments per row, ceil(nx / L)
  __host__ __device__ __forceinline__ size_t index(int i, int x, int y) const {
    return ((((size_t)y * (size_t)nseg + (size_t)(x >> lshift)) * 9 + (size_t)i) << lshift) +
           (size_t)(x & ((1 << lshift) - 1));
  }
  // doubles in one buffer (including padding lanes)
  __host__ __device__ __forceinline__ size_t size() const {
    return ((size_t)ny * (size_t)nseg * 9) << lshift;
  }
  // padded nodes (threads of a one-node-per-thread launch)
  __host__ __device__ __forceinline__ size_t padded_nodes() const {
    return ((size_t)ny * (size_t)nseg) << lshift;
  }
};

Geo make_geo(int nx, int ny);

// Arguments of one fused step launch.
struct StepArgs {
  const double* src;    // post-collision populations at t - 1 (device layout)
  double* dst;          // post-collision populations at t
  Geo g;
  int mode;             // 0 periodic, 1 pressure
  int shift;            // Eq. (20) specular source from x -/+ 1
  int xcd_remap;
  int ghost_lds;        // pressure mode: ghost columns staged in LDS (set by the launcher)
  double r;             // bounce-back fraction, Eq. (20)
  double gx, gy;        // body acceleration (periodic)
  int forcing;          // 1: source with the third-order force moments (see collide)
  double s3, snu, sq, s8;
  // pressure mode: per-column rates from the local Knudsen number
  double kn;            // Kn_out
  double a;             // Bosanquet factor
  double A2;            // B2
  double tq_den;        // denominator of Eq. (21)
  double c_tau;         // sqrt(6/pi) * N, N = ny
  double rho_in, rho_out;
  // pressure mode, large grids (row kernel): scratch filled by the prep kernel
  // each step; null when the caller provides none (column kernel only)
  double* col_rates;    // [2][nx]: s_nu(x), then s_q(x)
  double* ghosts;       // [2][9][ny]: inlet, outlet ghost columns
  int pressure_path;    // 0 by size, 1 column kernel, 2 row kernel
  int cus;              // compute units of the device (launch-shape choice; 0: unknown)
};
// Compute units of the current device (0 if the query fails).
int device_cus();

// Batch of pressure-driven channels on one grid (nx, ny, wall source shift
// shared): per-channel parameters of the step.
struct PChan {
  double r;             // bounce-back fraction, Eq. (20)
  double s3, s8;
  double kn, a, A2, tq_den;
  double rho_in, rho_out;
};

// Run state of one channel of such a batch.  Every channel starts at step 0
// in buffer 0; the channels still running share one step count and one
// current buffer, which the check kernel records in cur.
struct PChanState {
  int64_t steps;        // steps taken
  int32_t active;       // 0 once converged: no further steps
  int32_t have_prev;    // prev holds the mass flow of the previous check
  double prev;          // column-mean mass flow at the previous check
  int32_t cur;          // buffer holding the current populations
  int32_t pad;
};

struct PBatchArgs {
  double* buf[2];       // buffer k of channel c at buf[k] + c * stride
  size_t stride;        // doubles per channel buffer (Geo::size, padded)
  Geo g;
  int nch;              // step launches: channels in `live`; otherwise all channels
  const int32_t* live;  // [nch] indices of the channels a step launch covers
  int shift;            // Eq. (20) specular source from x -/+ 1
  int xcd_remap;
  int par;              // step: read buf[par], write buf[par ^ 1]
  int ghost_lds;        // set by the launcher
  int nblk;             // column workgroups per channel, set by the launcher
  int cus;
  double c_tau;         // sqrt(6/pi) * ny
  const PChan* ch;      // [nch]
  const PChanState* state;   // [nch]
  // row-kernel form: per-channel scratch filled by its prep launch each step
  // (null: column kernel only)
  double* col_rates;    // [nch][2][nx]
  double* ghosts;       // [nch][2][9][ny]
  int path;             // 0 by total size, 1 column kernel, 2 row kernel
};

struct InitArgs {
  double* dst;
  Geo g;
  int kind;             // clb_init_kind
  double rho0, ux0, uy0;
  double rho_in, rho_out;
  double amp;
  uint64_t seed;
};

struct DiagArgs {
  const double* src;
  Geo g;
  int mode;
  int shift;
  double r;
  double gx, gy;
  double rho_in, rho_out;
  double* rho;
  double* ux;
  double* uy;
  double* m;
  double* su;
  double* rhoc;
};

// Threads of periodic step workgroups allowed on one CU at a time.
constexpr int kStepThreadsPerCU = 1024;
// Pressure-mode grids with at least this many nodes take the row kernel
// (prep + row-streaming step) when the caller provides its scratch; below it
// the column kernel with wide workgroups is as fast or faster (measured).
constexpr size_t kPressureRowNodes = (size_t)1 << 21;
hipError_t periodic_step_lds(int block_x, size_t* bytes);
// lds_reserve: see periodic_step_lds (periodic mode only).
hipError_t launch_step(const StepArgs& a, int block_x, hipStream_t st, size_t lds_reserve = 0);
// Batches with at least this many nodes in all take the row kernel.
constexpr size_t kPBatchRowNodes = (size_t)1 << 21;
// One step of every active channel of a pressure-driven batch; lds_reserve
// as for launch_step (row kernel only).
hipError_t launch_pbatch_step(const PBatchArgs& a, hipStream_t st, size_t lds_reserve = 0);
// k = 2..4 steps of every active channel in one launch, where
// pbatch_multi_step_ok holds (ny <= 48, column-kernel path for the running
// channels); needs stepk_setup.
bool pbatch_multi_step_ok(const PBatchArgs& a);
hipError_t launch_pbatch_stepk(const PBatchArgs& a, int k, hipStream_t st);
// k = 2, 3 or 4 periodic or pressure-driven steps in one launch (a.src ->
// a.dst, the steps before the last kept in LDS); stepk_setup allows their
// LDS sizes (once per device, before the first such launch).
hipError_t stepk_setup();
hipError_t launch_stepk(const StepArgs& a, int k, hipStream_t st);
bool periodic_multi_step_ok(const StepArgs& a);   // nx >= 64
// Pressure-driven form; only where pressure_multi_step_ok holds (ny <= 48,
// column-kernel path).
bool pressure_multi_step_ok(const StepArgs& a);
hipError_t launch_stepk_pressure(const StepArgs& a, int k, hipStream_t st);
hipError_t launch_init(const InitArgs& a, hipStream_t st);
// Plain copy of n16 16-byte words (HBM ceiling probe).
hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t st);
hipError_t launch_moments(const DiagArgs& a, hipStream_t st);
hipError_t launch_column_sums(const DiagArgs& a, hipStream_t st);
// The same sums over populations in the ABI layout [9][ny][nx] (a.src and
// a.g.lshift / nseg unused; a.g.nx, a.g.ny give the grid).
hipError_t launch_column_sums_plane(const DiagArgs& a, const double* P, hipStream_t st);
hipError_t launch_mean(const double* v, int n, double* out, hipStream_t st);
hipError_t launch_pressure_dev(const double* rhoc, int nx, double rho_in, double rho_out, double* dp,
                               hipStream_t st);
hipError_t launch_nonfinite(const double* p, const Geo& g, double* partial, int nblocks, double* out,
                            hipStream_t st);
// Copy between the ABI layout [9][ny][nx] and the device layout.
hipError_t launch_export(const double* src, const Geo& g, double* out, hipStream_t st);
hipError_t launch_import(const double* in, const Geo& g, double* dst, hipStream_t st);

}  // namespace clb

// Host helpers defined in clb_api.cpp and used by every ABI translation unit.
#include "clb.h"

namespace clb {
clb_status set_error(clb_status st, const char* message);
clb_status validate_params(const clb_params* p, clb_derived* d);
clb_status check_device_ptr(const void* ptr, size_t bytes, const char* name);
}  // namespace clb
