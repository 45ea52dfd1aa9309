// Mass flow of caller-held populations with no device allocation at all: for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc).  The quantity is
// clb_massflow's (Section 3.2: m(x) = sum_y rho u_x of the pre-collision
// state, Eqs. 5, 12, 13, 20 and the x boundaries, and its column mean); the
// kernels are the ones clb_massflow runs.  Their scratch -- the per-column
// sums when the caller passes no column array, and the mean -- lives in a
// fixed device array of this library instead of a workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "clb.h"
#include "clb_internal.hpp"
#include "clb_trace.hpp"

namespace {

// Scratch of clb_massflow_noalloc: CLB_NOALLOC_MAX_NX per-column sums and one
// result slot, 256-byte aligned.  Each GPU holds its own copy until the
// process ends.
constexpr size_t kScratchDoubles = (size_t)CLB_NOALLOC_MAX_NX + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (host code must not pass the array's own name to a kernel: on the
// host it is only a stand-in for the symbol).
clb_status scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return clb::set_error(CLB_EHIP, "clb_massflow_noalloc: hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return clb::set_error(CLB_EHIP, "clb_massflow_noalloc: device index too large");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char msg[256];
      std::snprintf(msg, sizeof(msg), "clb_massflow_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
      return clb::set_error(CLB_EHIP, msg);
    }
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return CLB_OK;
}

}  // namespace

extern "C" {

clb_status clb_massflow_noalloc(const clb_params* p, const double* d_P, double* d_m_col, double* h_m_mean,
                                void* hip_stream) {
  const clb::TraceRange trace("clb_massflow_noalloc");
  clb_derived d;
  clb_status st = clb::validate_params(p, &d);
  if (st != CLB_OK) return st;
  if (p->nx > CLB_NOALLOC_MAX_NX) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "nx: %d columns exceed the fixed scratch of clb_massflow_noalloc (%d)", p->nx,
                  CLB_NOALLOC_MAX_NX);
    return clb::set_error(CLB_EINVAL, msg);
  }
  const size_t plane = (size_t)p->nx * (size_t)p->ny;
  if ((st = clb::check_device_ptr(d_P, 9 * plane * sizeof(double), "d_P")) != CLB_OK) return st;
  if (d_m_col && (st = clb::check_device_ptr(d_m_col, (size_t)p->nx * sizeof(double), "d_m_col")) != CLB_OK)
    return st;
  if (!d_m_col && !h_m_mean) return CLB_OK;
  double* sc = nullptr;
  if ((st = scratch_ptr(&sc)) != CLB_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);

  clb::DiagArgs a{};
  a.g = clb::make_geo(p->nx, p->ny);
  a.mode = p->xbc;
  a.shift = p->cbbsr_shift;
  a.r = d.r;
  a.gx = p->xbc == CLB_X_PERIODIC ? p->gx : 0.0;
  a.gy = p->xbc == CLB_X_PERIODIC ? p->gy : 0.0;
  a.rho_in = p->p_ratio * p->rho_out;
  a.rho_out = p->rho_out;
  a.m = d_m_col ? d_m_col : sc;
  double* result = sc + CLB_NOALLOC_MAX_NX;
  hipError_t e = clb::launch_column_sums_plane(a, d_P, stream);
  if (e == hipSuccess && h_m_mean) e = clb::launch_mean(a.m, p->nx, result, stream);
  if (e == hipSuccess && h_m_mean) e = hipMemcpyAsync(h_m_mean, result, sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && h_m_mean) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    char msg[256];
    std::snprintf(msg, sizeof(msg), "clb_massflow_noalloc: %s", hipGetErrorString(e));
    return clb::set_error(CLB_EHIP, msg);
  }
  return CLB_OK;
}

}  // extern "C"
