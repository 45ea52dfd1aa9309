// Internal declarations shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace clb {

// Arguments of one fused step launch.
struct StepArgs {
  const double* src;    // post-collision populations at t - 1, [9][ny][nx]
  double* dst;          // post-collision populations at t
  size_t plane;         // nx * ny
  int nx, ny;
  int nseg;             // row segments per row (periodic kernel)
  int mode;             // 0 periodic, 1 pressure
  int shift;            // Eq. (20) specular source from x -/+ 1
  int xcd_remap;
  double r;             // bounce-back fraction, Eq. (20)
  double gx, gy;        // body acceleration (periodic)
  double s3, snu, sq, s8;
  // pressure mode: per-column rates from the local Knudsen number
  double kn;            // Kn_out
  double a;             // Bosanquet factor
  double A2;            // B2
  double tq_den;        // denominator of Eq. (21)
  double c_tau;         // sqrt(6/pi) * N, N = ny
  double rho_in, rho_out;
};

struct InitArgs {
  double* dst;
  int nx, ny;
  int kind;             // clb_init_kind
  double rho0, ux0, uy0;
  double rho_in, rho_out;
  double amp;
  uint64_t seed;
};

struct DiagArgs {
  const double* src;
  size_t plane;
  int nx, ny;
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

hipError_t launch_step(const StepArgs& a, int block_x, hipStream_t st);
hipError_t launch_init(const InitArgs& a, hipStream_t st);
hipError_t launch_moments(const DiagArgs& a, hipStream_t st);
hipError_t launch_column_sums(const DiagArgs& a, hipStream_t st);
hipError_t launch_mean(const double* v, int n, double* out, hipStream_t st);
hipError_t launch_pressure_dev(const double* rhoc, int nx, double rho_in, double rho_out, double* dp,
                               hipStream_t st);
hipError_t launch_nonfinite(const double* p, size_t n, double* partial, int nblocks, double* out,
                            hipStream_t st);

}  // namespace clb
