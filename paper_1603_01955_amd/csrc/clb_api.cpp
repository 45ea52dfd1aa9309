// C ABI of the cascaded LB library (declared in include/clb.h).
//
// Host side only: parameter validation and derivation (Eqs. 14-18, 21 and
// the values of Section 3), workspace carving, launch dispatch on the
// caller's stream, and the diagnostics plumbing.  No device memory is
// allocated here: the caller's workspace holds every device buffer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "clb.h"
#include "clb_internal.hpp"
#include "clb_trace.hpp"

namespace {

thread_local char g_err[512] = "";

clb_status fail(clb_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

clb_status hip_fail(hipError_t e, const char* where) {
  return fail(CLB_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define CLB_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

constexpr double kPi = 3.14159265358979323846;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int kPartials = 1024;

struct Layout {
  size_t buf;      // bytes of one population buffer
  size_t col;      // bytes of one per-column array
  size_t ghosts;   // bytes of the ghost-column scratch [2][9][ny]
  size_t total;
};

Layout layout_of(const clb_params* p) {
  Layout L;
  const clb::Geo g = clb::make_geo(p->nx, p->ny);
  L.buf = align256(g.size() * sizeof(double));
  L.col = align256((size_t)p->nx * sizeof(double));
  L.ghosts = align256(18 * (size_t)p->ny * sizeof(double));
  // two buffers, four diagnostics columns, two rate columns, ghost scratch,
  // reduction partials, results
  L.total = 2 * L.buf + 6 * L.col + L.ghosts + align256(kPartials * sizeof(double)) +
            align256(32 * sizeof(double));
  return L;
}

bool finite(double v) { return std::isfinite(v); }

// Validate *p and fill *d.  Eqs. (18), (21); A1 and r from Section 3.
clb_status validate(const clb_params* p, clb_derived* d) {
  if (!p) return fail(CLB_EINVAL, "params: NULL");
  if (p->nx < 1) return fail(CLB_EINVAL, "nx: must be >= 1 (got %d)", p->nx);
  if (p->ny < 1) return fail(CLB_EINVAL, "ny: must be >= 1 (got %d)", p->ny);
  if (p->xbc != CLB_X_PERIODIC && p->xbc != CLB_X_PRESSURE)
    return fail(CLB_EINVAL, "xbc: unknown boundary kind %d", p->xbc);
  if (p->xbc == CLB_X_PRESSURE && p->nx < 2) return fail(CLB_EINVAL, "nx: pressure mode needs nx >= 2");
  if (p->init < CLB_INIT_UNIFORM || p->init > CLB_INIT_PERTURBED)
    return fail(CLB_EINVAL, "init: unknown kind %d", p->init);
  if (!(finite(p->kn) && p->kn > 0)) return fail(CLB_EINVAL, "kn: must be finite and > 0");
  if (!(finite(p->a) && p->a >= 0)) return fail(CLB_EINVAL, "a: must be finite and >= 0");
  if (!(finite(p->sigma) && p->sigma > 0 && p->sigma <= 2))
    return fail(CLB_EINVAL, "sigma: must lie in (0, 2]");
  if (!std::isnan(p->A1) && !(finite(p->A1) && p->A1 >= 0))
    return fail(CLB_EINVAL, "A1: must be NaN (derive from sigma) or finite and >= 0");
  if (!(finite(p->A2) && p->A2 >= 0)) return fail(CLB_EINVAL, "A2: must be finite and >= 0");
  if (!std::isnan(p->r) && !(p->r >= 0 && p->r <= 1))
    return fail(CLB_EINVAL, "r: must be NaN (derive from A1) or lie in [0, 1]");
  if (!(finite(p->s3) && p->s3 > 0 && p->s3 < 2)) return fail(CLB_EINVAL, "s3: must lie in (0, 2)");
  if (!(finite(p->s8) && p->s8 > 0 && p->s8 < 2)) return fail(CLB_EINVAL, "s8: must lie in (0, 2)");
  if (!(finite(p->gx) && finite(p->gy))) return fail(CLB_EINVAL, "gx/gy: must be finite");
  if (p->xbc == CLB_X_PRESSURE && (p->gx != 0 || p->gy != 0))
    return fail(CLB_EINVAL, "gx/gy: must be 0 in pressure mode");
  if (!(finite(p->p_ratio) && p->p_ratio > 0)) return fail(CLB_EINVAL, "p_ratio: must be finite and > 0");
  if (!(finite(p->rho_out) && p->rho_out > 0)) return fail(CLB_EINVAL, "rho_out: must be finite and > 0");
  if (!(finite(p->rho0) && p->rho0 > 0)) return fail(CLB_EINVAL, "rho0: must be finite and > 0");
  if (!(finite(p->ux0) && finite(p->uy0))) return fail(CLB_EINVAL, "ux0/uy0: must be finite");
  if (!(finite(p->init_amp) && p->init_amp >= 0)) return fail(CLB_EINVAL, "init_amp: must be finite and >= 0");
  if (!(finite(p->tq_den) && p->tq_den > 0)) return fail(CLB_EINVAL, "tq_den: must be finite and > 0");
  if (p->cbbsr_shift != 0 && p->cbbsr_shift != 1) return fail(CLB_EINVAL, "cbbsr_shift: must be 0 or 1");
  if (p->forcing != 0 && p->forcing != 1) return fail(CLB_EINVAL, "forcing: must be 0 or 1");
  // Launch-shape limit of the periodic kernel (64-thread blocks at worst).
  if (clb::make_geo(p->nx, p->ny).padded_nodes() / 64 >= ((size_t)1 << 31))
    return fail(CLB_EINVAL, "nx*ny: grid too large for one launch");

  clb_derived dd;
  dd.A1 = std::isnan(p->A1) ? (1.0 - 0.1817 * p->sigma) * (2.0 - p->sigma) / p->sigma : p->A1;
  dd.r = std::isnan(p->r) ? 1.0 / (1.0 + dd.A1 * std::sqrt(kPi / 6.0)) : p->r;
  dd.tau_tilde = std::sqrt(6.0 / kPi) * (double)p->ny * p->kn / (1.0 + p->a * p->kn);
  dd.s_nu = 1.0 / (0.5 + dd.tau_tilde);
  dd.s_q = 1.0 / (0.5 + (3.0 + 4.0 * kPi * dd.tau_tilde * dd.tau_tilde * p->A2) / (p->tq_den * dd.tau_tilde));
  if (!(dd.s_nu > 0 && dd.s_nu < 2 && dd.s_q > 0 && dd.s_q < 2 && finite(dd.r)))
    return fail(CLB_EINVAL, "kn/a/A2: derived relaxation rates out of (0, 2)");
  if (d) *d = dd;
  return CLB_OK;
}

// The pointer must be device memory and [ptr, ptr + bytes) must lie inside
// one allocation.
clb_status check_device_range(const void* ptr, size_t bytes, const char* name) {
  if (!ptr) return fail(CLB_EINVAL, "%s: NULL", name);
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CLB_EINVAL, "%s: not a device pointer (%s)", name, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice)
    return fail(CLB_EINVAL, "%s: not device memory", name);
  void* base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CLB_EINVAL, "%s: unknown allocation (%s)", name, hipGetErrorString(e));
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(ptr);
  if (q < b || (size_t)(q - b) + bytes > size)
    return fail(CLB_EINVAL, "%s: %zu bytes do not fit in the allocation", name, bytes);
  if (((uintptr_t)ptr & 7) != 0) return fail(CLB_EINVAL, "%s: must be 8-byte aligned", name);
  return CLB_OK;
}

}  // namespace

struct clb_ctx {
  clb_params p;
  clb_derived d;
  clb::Geo g;           // device layout of the population buffers
  double* buf[2];
  int cur;              // buf[cur] holds the current post-collision state
  double* col_m;
  double* col_su;
  double* col_rc;
  double* col_tmp;
  double* partial;
  double* result;
  hipStream_t stream;
  int64_t steps;
  int block_x;
  size_t step_lds;       // LDS reserved per row-streaming step workgroup (occupancy cap)
  int pressure_path;      // clb_set_pressure_path
  int cus;               // compute units of the device
  double* col_rates;     // pressure mode, large grids: per-column s_nu, s_q
  double* ghosts;        // pressure mode, large grids: ghost columns
  int xcd_remap;
  int steps_per_launch;  // steps per launch, 1-4 (those before the last kept in LDS)
  int64_t check_every;   // clb_step checks for non-finite populations at multiples of this step count (0: never)
  // optional hipGraph of graph_steps steps, one per starting buffer
  int graph_steps;
  int graph_flip;        // buffer parity change of one graph replay (launches mod 2)
  hipStream_t capture;  // private stream used only to record the graphs
  hipGraph_t graph[2];
  hipGraphExec_t gexec[2];
};

namespace {

clb::StepArgs step_args(const clb_ctx* c) {
  clb::StepArgs a{};
  a.src = c->buf[c->cur];
  a.dst = c->buf[c->cur ^ 1];
  a.g = c->g;
  a.mode = c->p.xbc;
  a.shift = c->p.cbbsr_shift;
  a.xcd_remap = c->xcd_remap;
  a.r = c->d.r;
  a.gx = c->p.gx;
  a.gy = c->p.gy;
  a.forcing = c->p.forcing;
  a.s3 = c->p.s3;
  a.snu = c->d.s_nu;
  a.sq = c->d.s_q;
  a.s8 = c->p.s8;
  a.kn = c->p.kn;
  a.a = c->p.a;
  a.A2 = c->p.A2;
  a.tq_den = c->p.tq_den;
  a.c_tau = std::sqrt(6.0 / kPi) * (double)c->p.ny;
  a.rho_in = c->p.p_ratio * c->p.rho_out;
  a.rho_out = c->p.rho_out;
  a.col_rates = c->col_rates;
  a.ghosts = c->ghosts;
  a.pressure_path = c->pressure_path;
  a.cus = c->cus;
  return a;
}

clb::DiagArgs diag_args(const clb_ctx* c) {
  clb::DiagArgs a{};
  a.src = c->buf[c->cur];
  a.g = c->g;
  a.mode = c->p.xbc;
  a.shift = c->p.cbbsr_shift;
  a.r = c->d.r;
  a.gx = c->p.gx;
  a.gy = c->p.gy;
  a.rho_in = c->p.p_ratio * c->p.rho_out;
  a.rho_out = c->p.rho_out;
  return a;
}

clb_status check_ctx(const clb_ctx* c) {
  if (!c) return fail(CLB_EINVAL, "ctx: NULL");
  return CLB_OK;
}

clb_status run_column_sums(clb_ctx* c, double* m, double* su, double* rc) {
  clb::DiagArgs a = diag_args(c);
  a.m = m;
  a.su = su;
  a.rhoc = rc;
  CLB_HIP(clb::launch_column_sums(a, c->stream));
  return CLB_OK;
}

clb_status read_result(clb_ctx* c, double* h) {
  CLB_HIP(hipMemcpyAsync(h, c->result, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CLB_HIP(hipStreamSynchronize(c->stream));
  return CLB_OK;
}

}  // namespace

extern "C" {

void clb_params_default(clb_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = 1;
  p->ny = 1;
  p->xbc = CLB_X_PERIODIC;
  p->init = CLB_INIT_UNIFORM;
  p->kn = 0.1;
  p->a = 2.0;        // Section 3
  p->sigma = 1.0;
  p->A1 = NAN;       // -> (1 - 0.1817 sigma)(2 - sigma)/sigma
  p->A2 = 0.55;      // Section 3
  p->r = NAN;        // -> Eq. (21)
  p->s3 = 1.1;       // Section 3
  p->s8 = 1.2;       // Section 3
  p->p_ratio = 2.0;
  p->rho_out = 1.0;
  p->rho0 = 1.0;
  p->tq_den = 16.0;  // Eq. (21) as printed
  p->cbbsr_shift = 1;
}

clb_status clb_derive(const clb_params* p, clb_derived* out) {
  if (!out) return fail(CLB_EINVAL, "out: NULL");
  return validate(p, out);
}

clb_status clb_workspace_size(const clb_params* p, size_t* bytes) {
  if (!bytes) return fail(CLB_EINVAL, "bytes: NULL");
  clb_status st = validate(p, nullptr);
  if (st != CLB_OK) return st;
  *bytes = layout_of(p).total;
  return CLB_OK;
}

clb_status clb_init(const clb_params* p, void* d_workspace, size_t bytes, void* hip_stream, clb_ctx** out) {
  const clb::TraceRange trace("clb_init");
  if (!out) return fail(CLB_EINVAL, "out: NULL");
  *out = nullptr;
  clb_derived d;
  clb_status st = validate(p, &d);
  if (st != CLB_OK) return st;
  const Layout L = layout_of(p);
  if (!d_workspace) return fail(CLB_EINVAL, "d_workspace: NULL");
  if (bytes < L.total) return fail(CLB_ENOMEM, "workspace: %zu bytes given, %zu needed", bytes, L.total);
  st = check_device_range(d_workspace, L.total, "d_workspace");
  if (st != CLB_OK) return st;
  clb_ctx* c = new (std::nothrow) clb_ctx();   // value-initialised: no graphs yet
  if (!c) return fail(CLB_ENOMEM, "host context allocation failed");
  c->p = *p;
  c->d = d;
  c->g = clb::make_geo(p->nx, p->ny);
  char* base = static_cast<char*>(d_workspace);
  c->buf[0] = reinterpret_cast<double*>(base);
  c->buf[1] = reinterpret_cast<double*>(base + L.buf);
  char* q = base + 2 * L.buf;
  c->col_m = reinterpret_cast<double*>(q);
  c->col_su = reinterpret_cast<double*>(q + L.col);
  c->col_rc = reinterpret_cast<double*>(q + 2 * L.col);
  c->col_tmp = reinterpret_cast<double*>(q + 3 * L.col);
  c->partial = reinterpret_cast<double*>(q + 4 * L.col);
  c->result = reinterpret_cast<double*>(q + 4 * L.col + align256(kPartials * sizeof(double)));
  q += 4 * L.col + align256(kPartials * sizeof(double)) + align256(32 * sizeof(double));
  c->col_rates = reinterpret_cast<double*>(q);   // [2][nx] (two columns of L.col bytes each)
  c->ghosts = reinterpret_cast<double*>(q + 2 * L.col);
  c->cur = 0;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  c->block_x = 1024;
  c->xcd_remap = 1;
  c->pressure_path = 0;
  c->cus = clb::device_cus();
  c->step_lds = 0;
  c->steps_per_launch = p->xbc == CLB_X_PERIODIC ? 3 : 4;
  {
    hipError_t e = clb::periodic_step_lds(c->block_x, &c->step_lds);
    if (e == hipSuccess) e = clb::stepk_setup();
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "clb_init: device attributes");
    }
  }

  clb::InitArgs ia{};
  ia.dst = c->buf[0];
  ia.g = c->g;
  ia.kind = p->init;
  ia.rho0 = p->rho0;
  ia.ux0 = p->ux0;
  ia.uy0 = p->uy0;
  ia.rho_in = p->p_ratio * p->rho_out;
  ia.rho_out = p->rho_out;
  ia.amp = p->init_amp;
  ia.seed = p->seed;
  hipError_t e = clb::launch_init(ia, c->stream);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "clb_init: init kernel");
  }
  *out = c;
  return CLB_OK;
}

}  // extern "C"

// Helpers of the stepping entry points.  They sit outside the extern "C"
// block: C language linkage would give them plain exported names, which any
// other loaded object defining the same name could take over at run time.
namespace {

void drop_graphs(clb_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
}

// Enqueue n steps on stream st starting from buffer parity *cur (updated):
// steps_per_launch steps per launch while that many remain, then the
// remainder in one launch, where the multi-step kernels apply (periodic
// mode: nx >= 64; pressure mode: at most 48 rows on the column path); else
// one per launch.
hipError_t enqueue_steps(const clb_ctx* c, int64_t n, hipStream_t st, int* cur) {
  const bool periodic = c->p.xbc == CLB_X_PERIODIC;
  int k = c->steps_per_launch;
  if (periodic && !clb::periodic_multi_step_ok(step_args(c))) k = 1;
  if (!periodic && !clb::pressure_multi_step_ok(step_args(c))) k = 1;
  hipError_t e = hipSuccess;
  while (n > 0 && e == hipSuccess) {
    clb::StepArgs a = step_args(c);
    a.src = c->buf[*cur];
    a.dst = c->buf[*cur ^ 1];
    const int m = n < k ? (int)n : k;
    if (m >= 2) {
      e = periodic ? clb::launch_stepk(a, m, st) : clb::launch_stepk_pressure(a, m, st);
      n -= m;
    } else {
      e = clb::launch_step(a, c->block_x, st, c->step_lds);
      n -= 1;
    }
    *cur ^= 1;
  }
  return e;
}

// Record graph_steps steps starting from buffer parity c->cur on the
// private capture stream (recording only: nothing runs there).
clb_status record_graph(clb_ctx* c) {
  const int p = c->cur;
  if (!c->capture) CLB_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  CLB_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
  int cur = p;
  const hipError_t e = enqueue_steps(c, c->graph_steps, c->capture, &cur);
  c->graph_flip = cur ^ p;
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->capture, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "step launch during graph capture");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  c->graph[p] = g;
  CLB_HIP(hipGraphInstantiate(&c->gexec[p], g, nullptr, nullptr, 0));
  return CLB_OK;
}

}  // namespace

namespace {

// Enqueue n >= 0 steps: hipGraph replays while whole graphs fit, then single
// launches.  Updates the buffer parity and the step counter.
clb_status advance(clb_ctx* c, int64_t n) {
  clb_status st = CLB_OK;
  while (c->graph_steps > 0 && n >= c->graph_steps) {
    if (!c->gexec[c->cur] && (st = record_graph(c)) != CLB_OK) return st;
    CLB_HIP(hipGraphLaunch(c->gexec[c->cur], c->stream));
    c->cur ^= c->graph_flip;
    c->steps += c->graph_steps;
    n -= c->graph_steps;
  }
  CLB_HIP(enqueue_steps(c, n, c->stream, &c->cur));
  c->steps += n;
  return CLB_OK;
}

// Number of non-finite populations of the current state (synchronises).
clb_status count_nonfinite(clb_ctx* c, double* bad) {
  const size_t n = (size_t)c->p.nx * c->p.ny;
  size_t nb = (n + 255) / 256;
  if (nb > (size_t)kPartials) nb = kPartials;
  CLB_HIP(clb::launch_nonfinite(c->buf[c->cur], c->g, c->partial, (int)nb, c->result, c->stream));
  return read_result(c, bad);
}

}  // namespace

extern "C" {

clb_status clb_step(clb_ctx* c, int64_t nsteps) {
  const clb::TraceRange trace("clb_step");
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (nsteps < 0) return fail(CLB_EINVAL, "nsteps: must be >= 0");
  if (c->check_every <= 0) return advance(c, nsteps);
  // Failure detection: stop at every multiple of check_every (counted from
  // the start) and look for non-finite populations before going on.
  while (nsteps > 0) {
    const int64_t to_check = c->check_every - c->steps % c->check_every;
    const int64_t m = nsteps < to_check ? nsteps : to_check;
    if ((st = advance(c, m)) != CLB_OK) return st;
    nsteps -= m;
    if (c->steps % c->check_every != 0) break;
    double bad = 0;
    if ((st = count_nonfinite(c, &bad)) != CLB_OK) return st;
    if (bad != 0.0)
      return fail(CLB_EUNSTABLE, "populations: %.0f non-finite values after step %lld", bad, (long long)c->steps);
  }
  return CLB_OK;
}

clb_status clb_steps_done(const clb_ctx* c, int64_t* h_steps) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (!h_steps) return fail(CLB_EINVAL, "h_steps: NULL");
  *h_steps = c->steps;
  return CLB_OK;
}

clb_status clb_moments(clb_ctx* c, double* d_rho, double* d_ux, double* d_uy) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  const size_t bytes = (size_t)c->p.nx * c->p.ny * sizeof(double);
  if (d_rho && (st = check_device_range(d_rho, bytes, "d_rho")) != CLB_OK) return st;
  if (d_ux && (st = check_device_range(d_ux, bytes, "d_ux")) != CLB_OK) return st;
  if (d_uy && (st = check_device_range(d_uy, bytes, "d_uy")) != CLB_OK) return st;
  if (!d_rho && !d_ux && !d_uy) return CLB_OK;
  clb::DiagArgs a = diag_args(c);
  a.rho = d_rho;
  a.ux = d_ux;
  a.uy = d_uy;
  CLB_HIP(clb::launch_moments(a, c->stream));
  return CLB_OK;
}

clb_status clb_column_sums(clb_ctx* c, double* d_m, double* d_su, double* d_rhoc) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  const size_t bytes = (size_t)c->p.nx * sizeof(double);
  if (d_m && (st = check_device_range(d_m, bytes, "d_m")) != CLB_OK) return st;
  if (d_su && (st = check_device_range(d_su, bytes, "d_su")) != CLB_OK) return st;
  if (d_rhoc && (st = check_device_range(d_rhoc, bytes, "d_rhoc")) != CLB_OK) return st;
  return run_column_sums(c, d_m ? d_m : c->col_m, d_su ? d_su : c->col_su, d_rhoc ? d_rhoc : c->col_rc);
}

clb_status clb_massflow(clb_ctx* c, double* d_m_col, double* h_m_mean) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (d_m_col && (st = check_device_range(d_m_col, (size_t)c->p.nx * sizeof(double), "d_m_col")) != CLB_OK)
    return st;
  double* m = d_m_col ? d_m_col : c->col_m;
  if ((st = run_column_sums(c, m, c->col_su, c->col_rc)) != CLB_OK) return st;
  if (!h_m_mean) return CLB_OK;
  CLB_HIP(clb::launch_mean(m, c->p.nx, c->result, c->stream));
  return read_result(c, h_m_mean);
}

clb_status clb_flow_rate(clb_ctx* c, double* h_Q) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (!h_Q) return fail(CLB_EINVAL, "h_Q: NULL");
  if (c->p.xbc != CLB_X_PERIODIC || c->p.gx == 0)
    return fail(CLB_ESTATE, "clb_flow_rate: needs periodic mode with gx != 0");
  if ((st = run_column_sums(c, c->col_m, c->col_su, c->col_rc)) != CLB_OK) return st;
  CLB_HIP(clb::launch_mean(c->col_su, c->p.nx, c->result, c->stream));
  double mean_su = 0;
  if ((st = read_result(c, &mean_su)) != CLB_OK) return st;
  const double H = (double)c->p.ny;
  *h_Q = mean_su * std::sqrt(6.0) / (3.0 * c->p.gx * H * H);
  return CLB_OK;
}

clb_status clb_pressure_deviation(clb_ctx* c, double* d_dp, double* d_rho_c) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (c->p.xbc != CLB_X_PRESSURE) return fail(CLB_ESTATE, "clb_pressure_deviation: pressure mode only");
  const size_t bytes = (size_t)c->p.nx * sizeof(double);
  if ((st = check_device_range(d_dp, bytes, "d_dp")) != CLB_OK) return st;
  if (d_rho_c && (st = check_device_range(d_rho_c, bytes, "d_rho_c")) != CLB_OK) return st;
  double* rc = d_rho_c ? d_rho_c : c->col_rc;
  if ((st = run_column_sums(c, c->col_m, c->col_su, rc)) != CLB_OK) return st;
  CLB_HIP(clb::launch_pressure_dev(rc, c->p.nx, c->p.p_ratio * c->p.rho_out, c->p.rho_out, d_dp, c->stream));
  return CLB_OK;
}

clb_status clb_get_populations(clb_ctx* c, double* d_out) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  const size_t bytes = 9 * (size_t)c->p.nx * c->p.ny * sizeof(double);
  if ((st = check_device_range(d_out, bytes, "d_out")) != CLB_OK) return st;
  CLB_HIP(clb::launch_export(c->buf[c->cur], c->g, d_out, c->stream));
  return CLB_OK;
}

clb_status clb_set_populations(clb_ctx* c, const double* d_in) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  const size_t bytes = 9 * (size_t)c->p.nx * c->p.ny * sizeof(double);
  if ((st = check_device_range(d_in, bytes, "d_in")) != CLB_OK) return st;
  CLB_HIP(clb::launch_import(d_in, c->g, c->buf[c->cur], c->stream));
  c->steps = 0;
  return CLB_OK;
}

clb_status clb_check_finite(clb_ctx* c, int32_t* h_ok) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (!h_ok) return fail(CLB_EINVAL, "h_ok: NULL");
  double bad = 0;
  if ((st = count_nonfinite(c, &bad)) != CLB_OK) return st;
  *h_ok = bad == 0.0 ? 1 : 0;
  if (!*h_ok) return fail(CLB_EUNSTABLE, "populations: %.0f non-finite values", bad);
  return CLB_OK;
}

clb_status clb_set_check_every(clb_ctx* c, int64_t check_every) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (check_every < 0) return fail(CLB_EINVAL, "check_every: must be >= 0");
  c->check_every = check_every;
  return CLB_OK;
}

clb_status clb_set_launch(clb_ctx* c, int32_t block_x, int32_t xcd_remap) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (block_x != 64 && block_x != 128 && block_x != 256 && block_x != 512 && block_x != 1024)
    return fail(CLB_EINVAL, "block_x: must be 64, 128, 256, 512 or 1024");
  if (xcd_remap != 0 && xcd_remap != 1) return fail(CLB_EINVAL, "xcd_remap: must be 0 or 1");
  if (c->g.padded_nodes() / block_x >= ((size_t)1 << 31)) return fail(CLB_EINVAL, "block_x: grid too large");
  if (block_x != c->block_x || xcd_remap != c->xcd_remap) {
    CLB_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
  }
  CLB_HIP(clb::periodic_step_lds(block_x, &c->step_lds));
  c->block_x = block_x;
  c->xcd_remap = xcd_remap;
  return CLB_OK;
}

clb_status clb_set_steps_per_launch(clb_ctx* c, int32_t steps) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (steps < 1 || steps > 4) return fail(CLB_EINVAL, "steps: must be 1, 2, 3 or 4");
  if (steps != c->steps_per_launch) {
    CLB_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
  }
  c->steps_per_launch = steps;
  return CLB_OK;
}

clb_status clb_set_pressure_path(clb_ctx* c, int32_t path) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (path < 0 || path > 2) return fail(CLB_EINVAL, "path: must be 0, 1 or 2");
  if (path != c->pressure_path) {
    CLB_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
  }
  c->pressure_path = path;
  return CLB_OK;
}

clb_status clb_set_graph_steps(clb_ctx* c, int32_t steps_per_graph) {
  clb_status st = check_ctx(c);
  if (st != CLB_OK) return st;
  if (steps_per_graph < 0 || steps_per_graph > 100000)
    return fail(CLB_EINVAL, "steps_per_graph: must lie in [0, 100000]");
  if (steps_per_graph != c->graph_steps) {
    CLB_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->graph_steps = steps_per_graph;
  }
  return CLB_OK;
}

clb_status clb_destroy(clb_ctx* c) {
  if (!c) return fail(CLB_EINVAL, "ctx: NULL");
  if (c->gexec[0] || c->gexec[1]) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
  return CLB_OK;
}

clb_status clb_hbm_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream) {
  if (bytes % 16 != 0) return fail(CLB_EINVAL, "bytes: %zu is not a multiple of 16", bytes);
  if (!d_src || !d_dst) return fail(CLB_EINVAL, "d_src / d_dst: NULL");
  if (((uintptr_t)d_src & 15) != 0 || ((uintptr_t)d_dst & 15) != 0)
    return fail(CLB_EINVAL, "d_src / d_dst: must be 16-byte aligned");
  if (bytes == 0) return CLB_OK;
  if (bytes / 16 / 256 >= ((size_t)1 << 31)) return fail(CLB_EINVAL, "bytes: %zu too large for one launch", bytes);
  clb_status st = check_device_range(d_src, bytes, "d_src");
  if (st != CLB_OK) return st;
  if ((st = check_device_range(d_dst, bytes, "d_dst")) != CLB_OK) return st;
  const uintptr_t s0 = (uintptr_t)d_src, t0 = (uintptr_t)d_dst;
  if (s0 < t0 + bytes && t0 < s0 + bytes) return fail(CLB_EINVAL, "d_src / d_dst: ranges overlap");
  CLB_HIP(clb::launch_copy16(d_src, d_dst, bytes / 16, static_cast<hipStream_t>(hip_stream)));
  return CLB_OK;
}

const char* clb_last_error(void) { return g_err; }

}  // extern "C"

// Helpers shared with the other translation units of the library.
namespace clb {

clb_status set_error(clb_status st, const char* message) { return fail(st, "%s", message); }

clb_status validate_params(const clb_params* p, clb_derived* d) { return validate(p, d); }

clb_status check_device_ptr(const void* ptr, size_t bytes, const char* name) {
  return check_device_range(ptr, bytes, name);
}

}  // namespace clb
