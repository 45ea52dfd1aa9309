// Batch of pressure-driven long channels on one grid: the mass-flow sweep
// of Section 3.2 (dimensionless mass flow S = m / m_ns against Kn_out at a
// fixed pressure ratio and TMAC).
//
// Method: Liu & He, arXiv:1603.01955, Section 3.2.  Every channel has the
// same nx x ny grid and its own Kn_out, pressure ratio, outlet density, slip
// coefficients and rates.  One launch advances all channels that are still
// running (the column kernel, channel-major workgroups), so a sweep of many
// channels of the paper's size (a few hundred columns' worth of workgroups
// each) fills the chip where one channel alone cannot.  Convergence is
// checked on the device every check_every steps from the column-mean mass
// flow; the chunk of steps plus its check is recorded once as a hipGraph
// and replayed.  A channel advances bitwise as a single-channel context with
// the same parameters does.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "clb.h"
#include "clb_device.hpp"
#include "clb_gather.hpp"
#include "clb_internal.hpp"
#include "clb_trace.hpp"

namespace clb {
namespace {

constexpr int kMassThreads = 1024;

// Column-mean mass flow (1/nx) sum_x sum_y rho u_x of one channel's
// pre-collision state (Eqs. 5, 12, 13, 20 and the ghost columns), summed
// in a fixed order by one workgroup of kMassThreads threads: each thread
// walks whole columns, the threads' totals are added by wavefront
// butterflies and the wavefront totals in order.
__device__ double channel_massflow(const PBatchArgs& p, const PChan& ch, const double* P, double* s_red) {
  const Gather<1, View> gat{{P, p.g}, ch.r, 1.0 - ch.r, p.shift, ch.rho_in, ch.rho_out};
  double acc = 0.0;
  for (int x = threadIdx.x; x < p.g.nx; x += kMassThreads) {
    double m = 0.0;
    for (int y = 0; y < p.g.ny; ++y) {
      double f[9];
      gather_node(gat, x, y, f);
      double rho, ux, uy;
      rho_u(f, rho, ux, uy);
      m += rho * ux;
    }
    acc += m;
  }
  // wavefront sums, then the wavefront totals in order
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double m = s_red[0];
#pragma unroll
  for (int k = 1; k < kMassThreads / 64; ++k) m += s_red[k];
  return m / (double)p.g.nx;
}

// After `add` steps of the running channels, whose state is now in buffer
// `cur`: count them, record the buffer, and with `check` compare each running
// channel's mass flow with its previous check; the channel stops once
// |m - m_prev| <= tol |m|.  One workgroup per channel.
__global__ __launch_bounds__(kMassThreads) void k_pbatch_check(PBatchArgs p, PChanState* st, int add, int cur,
                                                                int check, double tol) {
  __shared__ double s_red[kMassThreads / 64];
  const int c = blockIdx.x;
  PChanState s = st[c];
  __syncthreads();   // every thread has read st[c] before thread 0 rewrites it
  if (!s.active) return;
  s.steps += add;
  s.cur = cur;
  if (check) {
    const double m = channel_massflow(p, p.ch[c], p.buf[s.cur] + (size_t)c * p.stride, s_red);
    if (s.have_prev && fabs(m - s.prev) <= tol * fabs(m)) s.active = 0;
    s.prev = m;
    s.have_prev = 1;
  }
  if (threadIdx.x == 0) st[c] = s;
}

// Mass flow of every channel's current state into m[nch].
__global__ __launch_bounds__(kMassThreads) void k_pbatch_mass(PBatchArgs p, const PChanState* st, double* m) {
  __shared__ double s_red[kMassThreads / 64];
  const int c = blockIdx.x;
  const double v = channel_massflow(p, p.ch[c], p.buf[st[c].cur] + (size_t)c * p.stride, s_red);
  if (threadIdx.x == 0) m[c] = v;
}

__global__ void k_pbatch_reset(PChanState* st, int nch) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nch) st[c] = PChanState{0, 1, 0, 0.0, 0, 0};
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int kPartials = 1024;   // reduction partials of the finiteness check

struct PBatchLayout {
  size_t buf;     // bytes of one channel buffer
  size_t col;     // bytes of one per-column array
  size_t rates;   // bytes of the row kernel's per-column rates, all channels
  size_t ghosts;  // bytes of the row kernel's ghost columns, all channels
  size_t total;
};

PBatchLayout pbatch_layout(int32_t nch, const clb_params& p) {
  PBatchLayout L{};
  L.buf = align256(make_geo(p.nx, p.ny).size() * sizeof(double));
  L.col = align256((size_t)p.nx * sizeof(double));
  L.rates = align256((size_t)nch * 2 * p.nx * sizeof(double));
  L.ghosts = align256((size_t)nch * 18 * p.ny * sizeof(double));
  // two buffers per channel, channel table, run states, mass flows, three
  // per-column diagnostics arrays, row-kernel scratch, running-channel list
  L.total = 2 * (size_t)nch * L.buf + align256(nch * sizeof(PChan)) + align256(nch * sizeof(PChanState)) +
            align256(nch * sizeof(double)) + 3 * L.col + L.rates + L.ghosts + align256(nch * sizeof(int32_t)) +
            align256(kPartials * sizeof(double)) + align256(nch * sizeof(double));
  return L;
}

#define PBATCH_HIP(call)                                                   \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      char m_[256];                                                        \
      snprintf(m_, sizeof(m_), "%s: %s", #call, hipGetErrorString(e_));    \
      return clb::set_error(CLB_EHIP, m_);                                 \
    }                                                                      \
  } while (0)

clb_status perr(clb_status st, const char* msg) { return set_error(st, msg); }

}  // namespace
}  // namespace clb

struct clb_pbatch {
  int32_t nch;
  std::vector<clb_params> p;
  std::vector<clb::PChan> chan;            // host copy of the channel table
  clb::PBatchArgs args;                    // par is set per launch
  clb::PChanState* d_state;
  double* d_m;
  double* col[3];                          // per-column diagnostics scratch
  std::vector<clb::PChanState> h_state;    // mirror of d_state, current after every call
  std::vector<double> h_m;
  int32_t* d_live;                         // indices of the running channels (step launches)
  double* d_partial;                       // finiteness check: reduction partials and per-channel counts
  double* d_bad;
  std::vector<int32_t> h_live;             // host copy, read by the last upload
  int32_t n_live;
  int64_t t;                               // steps taken by the channels still running
  int32_t par;                             // buffer holding their current state
  int32_t steps_per_launch;                // 2-4: multi-step launches where they apply, 1: one step
  hipStream_t stream;                      // caller's stream: all work runs here
  hipStream_t capture;                     // private stream, used only to record graphs
  size_t step_lds;                         // LDS reserved per row-kernel workgroup (occupancy cap)
  hipGraph_t graph[2];                     // check_every steps + check, per starting buffer
  hipGraphExec_t exec[2];
  int32_t g_end[2];                        // buffer after a replay, per starting buffer
  int32_t g_every;
  double g_tol;
  int32_t g_live;                          // running channels the graphs were recorded for
};

namespace {

const double kPi = 3.14159265358979323846;

void drop_graphs(clb_pbatch* b) {
  for (int k = 0; k < 2; ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    b->exec[k] = nullptr;
    b->graph[k] = nullptr;
  }
}

// n steps of the running channels from buffer *par (updated) --
// steps_per_launch per launch where the multi-step kernel applies, a shorter
// remainder in one launch -- then the count (and with check the
// convergence test) on stream st.
clb_status enqueue_chunk(clb_pbatch* b, hipStream_t st, int* par, int64_t n, int check, double tol) {
  clb::PBatchArgs a = b->args;
  a.nch = b->n_live;
  const int k = b->n_live > 0 && clb::pbatch_multi_step_ok(a) ? b->steps_per_launch : 1;
  for (int64_t left = n; left > 0 && b->n_live > 0;) {
    a.par = *par;
    const int m = left < k ? (int)left : k;
    if (m >= 2) {
      PBATCH_HIP(clb::launch_pbatch_stepk(a, m, st));
      left -= m;
    } else {
      PBATCH_HIP(clb::launch_pbatch_step(a, st, b->step_lds));
      left -= 1;
    }
    *par ^= 1;
  }
  clb::k_pbatch_check<<<b->nch, clb::kMassThreads, 0, st>>>(b->args, b->d_state, (int)n, *par, check, tol);
  PBATCH_HIP(hipGetLastError());
  return CLB_OK;
}

clb_status record_chunk(clb_pbatch* b, int par, int32_t every, double tol) {
  PBATCH_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  int end = par;
  clb_status st = enqueue_chunk(b, b->capture, &end, every, 1, tol);
  b->g_end[par] = end;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->capture, &g);
  if (st != CLB_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  PBATCH_HIP(e);
  b->graph[par] = g;
  PBATCH_HIP(hipGraphInstantiate(&b->exec[par], g, nullptr, nullptr, 0));
  return CLB_OK;
}

// Refresh the host mirror of the run states and, when channels have stopped,
// the list of running channels that step launches cover (upload finished
// before returning, so the host copy may change afterwards).
clb_status read_state(clb_pbatch* b) {
  PBATCH_HIP(hipMemcpyAsync(b->h_state.data(), b->d_state, b->nch * sizeof(clb::PChanState),
                            hipMemcpyDeviceToHost, b->stream));
  PBATCH_HIP(hipStreamSynchronize(b->stream));
  int32_t n = 0;
  for (int c = 0; c < b->nch; ++c)
    if (b->h_state[c].active) b->h_live[n++] = c;
  if (n != b->n_live) {
    b->n_live = n;
    if (n > 0) {
      PBATCH_HIP(hipMemcpyAsync(b->d_live, b->h_live.data(), n * sizeof(int32_t), hipMemcpyHostToDevice,
                                b->stream));
      PBATCH_HIP(hipStreamSynchronize(b->stream));
    }
  }
  return CLB_OK;
}

// Diagnostics arguments for channel ch's current state.
clb::DiagArgs diag_of(const clb_pbatch* b, int ch) {
  const clb::PChan& c = b->chan[ch];
  clb::DiagArgs d{};
  d.src = b->args.buf[b->h_state[ch].cur] + (size_t)ch * b->args.stride;
  d.g = b->args.g;
  d.mode = CLB_X_PRESSURE;
  d.shift = b->args.shift;
  d.r = c.r;
  d.rho_in = c.rho_in;
  d.rho_out = c.rho_out;
  return d;
}

clb_status check_ch(const clb_pbatch* b, int32_t ch) {
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (ch < 0 || ch >= b->nch) return clb::perr(CLB_EINVAL, "ch: out of range");
  return CLB_OK;
}

}  // namespace

extern "C" {

clb_status clb_pbatch_workspace_size(int32_t nch, const clb_params* params, size_t* bytes) {
  if (!bytes) return clb::perr(CLB_EINVAL, "bytes: NULL");
  if (nch < 1 || !params) return clb::perr(CLB_EINVAL, "nch/params: need at least one channel");
  for (int c = 0; c < nch; ++c) {
    clb_status st = clb::validate_params(&params[c], nullptr);
    if (st != CLB_OK) return st;
    if (params[c].xbc != CLB_X_PRESSURE) return clb::perr(CLB_EINVAL, "xbc: every channel must be pressure-driven");
    if (params[c].nx != params[0].nx || params[c].ny != params[0].ny)
      return clb::perr(CLB_EINVAL, "nx/ny: every channel must have the same grid");
    if (params[c].cbbsr_shift != params[0].cbbsr_shift)
      return clb::perr(CLB_EINVAL, "cbbsr_shift: must be the same for every channel");
  }
  const size_t per_chan = 2 * clb::make_geo(params[0].nx, params[0].ny).size();
  if ((size_t)nch * per_chan / 2 >= ((size_t)1 << 40))
    return clb::perr(CLB_EINVAL, "nch*nx*ny: batch too large");
  *bytes = clb::pbatch_layout(nch, params[0]).total;
  return CLB_OK;
}

clb_status clb_pbatch_init(int32_t nch, const clb_params* params, void* d_workspace, size_t bytes, void* hip_stream,
                           clb_pbatch** out) {
  const clb::TraceRange trace("clb_pbatch_init");
  if (!out) return clb::perr(CLB_EINVAL, "out: NULL");
  *out = nullptr;
  size_t need = 0;
  clb_status st = clb_pbatch_workspace_size(nch, params, &need);
  if (st != CLB_OK) return st;
  if (!d_workspace) return clb::perr(CLB_EINVAL, "d_workspace: NULL");
  if (bytes < need) return clb::perr(CLB_ENOMEM, "workspace: smaller than clb_pbatch_workspace_size");
  if ((st = clb::check_device_ptr(d_workspace, need, "d_workspace")) != CLB_OK) return st;
  const clb::Geo g = clb::make_geo(params[0].nx, params[0].ny);
  // launch-shape limits: below 2^31 workgroups in the column kernel (at least
  // 4 columns per workgroup) and in the row kernel (1024 nodes each)
  if ((size_t)nch * (size_t)((g.nx + 3) / 4) >= ((size_t)1 << 31) ||
      (size_t)nch * ((g.padded_nodes() + 1023) / 1024) >= ((size_t)1 << 31))
    return clb::perr(CLB_EINVAL, "nch*nx*ny: too many workgroups for one launch");

  clb_pbatch* b = new (std::nothrow) clb_pbatch();
  if (!b) return clb::perr(CLB_ENOMEM, "host context allocation failed");
  b->nch = nch;
  b->p.assign(params, params + nch);
  for (int c = 0; c < nch; ++c) {
    const clb_params& p = params[c];
    clb_derived d;
    clb::validate_params(&p, &d);
    clb::PChan ch{};
    ch.r = d.r;
    ch.s3 = p.s3;
    ch.s8 = p.s8;
    ch.kn = p.kn;
    ch.a = p.a;
    ch.A2 = p.A2;
    ch.tq_den = p.tq_den;
    ch.rho_in = p.p_ratio * p.rho_out;
    ch.rho_out = p.rho_out;
    b->chan.push_back(ch);
  }
  const clb::PBatchLayout L = clb::pbatch_layout(nch, params[0]);
  char* q = static_cast<char*>(d_workspace);
  clb::PBatchArgs& a = b->args;
  a.buf[0] = reinterpret_cast<double*>(q);
  a.buf[1] = reinterpret_cast<double*>(q + (size_t)nch * L.buf);
  q += 2 * (size_t)nch * L.buf;
  a.stride = L.buf / sizeof(double);
  a.g = g;
  a.nch = nch;
  a.shift = params[0].cbbsr_shift;
  a.xcd_remap = 1;
  a.par = 0;
  a.cus = clb::device_cus();
  a.c_tau = std::sqrt(6.0 / kPi) * (double)params[0].ny;
  clb::PChan* d_ch = reinterpret_cast<clb::PChan*>(q);
  a.ch = d_ch;
  q += clb::align256(nch * sizeof(clb::PChan));
  b->d_state = reinterpret_cast<clb::PChanState*>(q);
  a.state = b->d_state;
  q += clb::align256(nch * sizeof(clb::PChanState));
  b->d_m = reinterpret_cast<double*>(q);
  q += clb::align256(nch * sizeof(double));
  for (int k = 0; k < 3; ++k) b->col[k] = reinterpret_cast<double*>(q + k * L.col);
  q += 3 * L.col;
  a.col_rates = reinterpret_cast<double*>(q);
  a.ghosts = reinterpret_cast<double*>(q + L.rates);
  q += L.rates + L.ghosts;
  a.path = 0;
  b->d_live = reinterpret_cast<int32_t*>(q);
  q += clb::align256(nch * sizeof(int32_t));
  b->d_partial = reinterpret_cast<double*>(q);
  b->d_bad = reinterpret_cast<double*>(q + clb::align256(clb::kPartials * sizeof(double)));
  a.live = b->d_live;
  b->h_live.resize(nch);
  for (int c = 0; c < nch; ++c) b->h_live[c] = c;
  b->n_live = nch;
  b->h_state.assign(nch, clb::PChanState{0, 1, 0, 0.0, 0, 0});
  b->h_m.assign(nch, 0.0);
  b->t = 0;
  b->par = 0;
  b->steps_per_launch = 4;
  b->stream = static_cast<hipStream_t>(hip_stream);

  auto fail_init = [b](hipError_t e, const char* where) {
    char m[256];
    snprintf(m, sizeof(m), "%s: %s", where, hipGetErrorString(e));
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return clb::set_error(CLB_EHIP, m);
  };
  hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e != hipSuccess) return fail_init(e, "hipStreamCreateWithFlags");
  e = clb::periodic_step_lds(1024, &b->step_lds);
  if (e == hipSuccess) e = clb::stepk_setup();
  if (e != hipSuccess) return fail_init(e, "device attributes");
  e = hipMemcpyAsync(d_ch, b->chan.data(), nch * sizeof(clb::PChan), hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return fail_init(e, "upload channel table");
  e = hipMemcpyAsync(b->d_live, b->h_live.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return fail_init(e, "upload channel list");
  for (int c = 0; c < nch && e == hipSuccess; ++c) {
    const clb_params& p = params[c];
    clb::InitArgs ia{};
    ia.dst = a.buf[0] + (size_t)c * a.stride;
    ia.g = g;
    ia.kind = p.init;
    ia.rho0 = p.rho0;
    ia.ux0 = p.ux0;
    ia.uy0 = p.uy0;
    ia.rho_in = p.p_ratio * p.rho_out;
    ia.rho_out = p.rho_out;
    ia.amp = p.init_amp;
    ia.seed = p.seed;
    e = clb::launch_init(ia, b->stream);
  }
  if (e != hipSuccess) return fail_init(e, "init kernel");
  clb::k_pbatch_reset<<<(nch + 255) / 256, 256, 0, b->stream>>>(b->d_state, nch);
  e = hipGetLastError();
  if (e != hipSuccess) return fail_init(e, "state reset kernel");
  // The uploads read b->chan and b->h_live; finish them before returning.
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail_init(e, "hipStreamSynchronize");
  *out = b;
  return CLB_OK;
}

clb_status clb_pbatch_step(clb_pbatch* b, int64_t nsteps) {
  const clb::TraceRange trace("clb_pbatch_step");
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (nsteps < 0) return clb::perr(CLB_EINVAL, "nsteps: must be >= 0");
  if (nsteps == 0) return CLB_OK;
  clb_status st = enqueue_chunk(b, b->stream, &b->par, nsteps, 0, 0.0);
  if (st != CLB_OK) return st;
  b->t += nsteps;
  for (auto& s : b->h_state)
    if (s.active) {
      s.steps += nsteps;
      s.cur = b->par;
    }
  return CLB_OK;
}

clb_status clb_pbatch_run(clb_pbatch* b, int64_t max_steps, int32_t check_every, double tol, int64_t* h_steps,
                          int32_t* h_converged) {
  const clb::TraceRange trace("clb_pbatch_run");
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (max_steps < 0) return clb::perr(CLB_EINVAL, "max_steps: must be >= 0");
  if (check_every < 0 || check_every > 100000) return clb::perr(CLB_EINVAL, "check_every: must lie in [0, 100000]");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return clb::perr(CLB_EINVAL, "tol: must be finite and >= 0");
  clb_status st = CLB_OK;
  if (check_every == 0) {
    if ((st = clb_pbatch_step(b, max_steps)) != CLB_OK) return st;
  } else {
    if (b->g_every != check_every || b->g_tol != tol) {
      PBATCH_HIP(hipStreamSynchronize(b->stream));
      drop_graphs(b);
      b->g_every = check_every;
      b->g_tol = tol;
    }
    int64_t left = max_steps;
    while (left > 0 && b->n_live > 0) {
      if (b->g_live != b->n_live) {   // the graphs cover a fixed set of running channels
        drop_graphs(b);
        b->g_live = b->n_live;
      }
      const int par = b->par;
      const int64_t n = left < check_every ? left : check_every;
      if (n == check_every) {
        if (!b->exec[par] && (st = record_chunk(b, par, check_every, tol)) != CLB_OK) return st;
        PBATCH_HIP(hipGraphLaunch(b->exec[par], b->stream));
        b->par = b->g_end[par];
      } else if ((st = enqueue_chunk(b, b->stream, &b->par, n, 0, 0.0)) != CLB_OK) {
        return st;
      }
      b->t += n;
      left -= n;
      if ((st = read_state(b)) != CLB_OK) return st;
    }
  }
  if (h_steps || h_converged) {
    if ((st = read_state(b)) != CLB_OK) return st;
    for (int c = 0; c < b->nch; ++c) {
      if (h_steps) h_steps[c] = b->h_state[c].steps;
      if (h_converged) h_converged[c] = b->h_state[c].active ? 0 : 1;
    }
  }
  return CLB_OK;
}

clb_status clb_pbatch_set_steps_per_launch(clb_pbatch* b, int32_t steps) {
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (steps < 1 || steps > 4) return clb::perr(CLB_EINVAL, "steps: must be 1, 2, 3 or 4");
  if (steps != b->steps_per_launch) {
    PBATCH_HIP(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->steps_per_launch = steps;
  }
  return CLB_OK;
}

clb_status clb_pbatch_set_path(clb_pbatch* b, int32_t path) {
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (path < 0 || path > 2) return clb::perr(CLB_EINVAL, "path: must be 0, 1 or 2");
  if (path != b->args.path) {
    PBATCH_HIP(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->args.path = path;
  }
  return CLB_OK;
}

clb_status clb_pbatch_massflow(clb_pbatch* b, double* h_m, double* h_m_ns) {
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (!h_m && !h_m_ns) return clb::perr(CLB_EINVAL, "h_m/h_m_ns: both NULL");
  if (h_m) {
    clb::k_pbatch_mass<<<b->nch, clb::kMassThreads, 0, b->stream>>>(b->args, b->d_state, b->d_m);
    PBATCH_HIP(hipGetLastError());
    PBATCH_HIP(hipMemcpyAsync(b->h_m.data(), b->d_m, b->nch * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    PBATCH_HIP(hipStreamSynchronize(b->stream));
    for (int c = 0; c < b->nch; ++c) h_m[c] = b->h_m[c];
  }
  if (h_m_ns) {
    for (int c = 0; c < b->nch; ++c) {
      // Continuum no-slip mass flow of the long channel (isothermal,
      // lubrication limit): m = H^3 (p_in^2 - p_out^2) / (24 mu RT L) with
      // RT = 1/3, p = rho/3, H = ny, L = nx and the gas viscosity of
      // Eqs. (15)-(17) without the Bosanquet factor,
      // mu = (1/3) sqrt(6/pi) rho Kn H = (1/3) sqrt(6/pi) rho_out Kn_out H.
      const clb_params& p = b->p[c];
      const double H = (double)p.ny, L = (double)p.nx;
      const double p_out = p.rho_out / 3.0, p_in = p.p_ratio * p_out;
      const double mu = std::sqrt(6.0 / kPi) * p.rho_out * p.kn * H / 3.0;
      h_m_ns[c] = H * H * H * (p_in * p_in - p_out * p_out) / (8.0 * mu * L);
    }
  }
  return CLB_OK;
}

clb_status clb_pbatch_column_sums(clb_pbatch* b, int32_t ch, double* d_m, double* d_su, double* d_rhoc) {
  clb_status st = check_ch(b, ch);
  if (st != CLB_OK) return st;
  const size_t bytes = (size_t)b->args.g.nx * sizeof(double);
  if (d_m && (st = clb::check_device_ptr(d_m, bytes, "d_m")) != CLB_OK) return st;
  if (d_su && (st = clb::check_device_ptr(d_su, bytes, "d_su")) != CLB_OK) return st;
  if (d_rhoc && (st = clb::check_device_ptr(d_rhoc, bytes, "d_rhoc")) != CLB_OK) return st;
  clb::DiagArgs d = diag_of(b, ch);
  d.m = d_m ? d_m : b->col[0];
  d.su = d_su ? d_su : b->col[1];
  d.rhoc = d_rhoc ? d_rhoc : b->col[2];
  PBATCH_HIP(clb::launch_column_sums(d, b->stream));
  return CLB_OK;
}

clb_status clb_pbatch_pressure_deviation(clb_pbatch* b, int32_t ch, double* d_dp) {
  clb_status st = check_ch(b, ch);
  if (st != CLB_OK) return st;
  if ((st = clb::check_device_ptr(d_dp, (size_t)b->args.g.nx * sizeof(double), "d_dp")) != CLB_OK) return st;
  clb::DiagArgs d = diag_of(b, ch);
  d.m = b->col[0];
  d.su = b->col[1];
  d.rhoc = b->col[2];
  PBATCH_HIP(clb::launch_column_sums(d, b->stream));
  PBATCH_HIP(clb::launch_pressure_dev(b->col[2], b->args.g.nx, b->chan[ch].rho_in, b->chan[ch].rho_out, d_dp,
                                      b->stream));
  return CLB_OK;
}

clb_status clb_pbatch_get_populations(clb_pbatch* b, int32_t ch, double* d_out) {
  clb_status st = check_ch(b, ch);
  if (st != CLB_OK) return st;
  const size_t bytes = 9 * (size_t)b->args.g.nx * b->args.g.ny * sizeof(double);
  if ((st = clb::check_device_ptr(d_out, bytes, "d_out")) != CLB_OK) return st;
  PBATCH_HIP(clb::launch_export(diag_of(b, ch).src, b->args.g, d_out, b->stream));
  return CLB_OK;
}

clb_status clb_pbatch_set_populations(clb_pbatch* b, int32_t ch, const double* d_in) {
  clb_status st = check_ch(b, ch);
  if (st != CLB_OK) return st;
  const size_t bytes = 9 * (size_t)b->args.g.nx * b->args.g.ny * sizeof(double);
  if ((st = clb::check_device_ptr(d_in, bytes, "d_in")) != CLB_OK) return st;
  PBATCH_HIP(clb::launch_import(d_in, b->args.g, const_cast<double*>(diag_of(b, ch).src), b->stream));
  return CLB_OK;
}

clb_status clb_pbatch_check_finite(clb_pbatch* b, int32_t* h_ok) {
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  if (!h_ok) return clb::perr(CLB_EINVAL, "h_ok: NULL");
  const clb::Geo& g = b->args.g;
  size_t nb = ((size_t)g.nx * g.ny + 255) / 256;
  if (nb > (size_t)clb::kPartials) nb = clb::kPartials;
  for (int c = 0; c < b->nch; ++c)
    PBATCH_HIP(clb::launch_nonfinite(diag_of(b, c).src, g, b->d_partial, (int)nb, b->d_bad + c, b->stream));
  PBATCH_HIP(hipMemcpyAsync(b->h_m.data(), b->d_bad, b->nch * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  PBATCH_HIP(hipStreamSynchronize(b->stream));
  int bad = 0;
  for (int c = 0; c < b->nch; ++c) {
    h_ok[c] = b->h_m[c] == 0.0 ? 1 : 0;
    bad += !h_ok[c];
  }
  if (bad) {
    char m[128];
    snprintf(m, sizeof(m), "populations: %d channel(s) with non-finite values", bad);
    return clb::perr(CLB_EUNSTABLE, m);
  }
  return CLB_OK;
}

clb_status clb_pbatch_destroy(clb_pbatch* b) {
  if (!b) return clb::perr(CLB_EINVAL, "batch: NULL");
  (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
  return CLB_OK;
}

}  // extern "C"
