// Batched form of the CLB step for Kn sweeps (many small periodic channels).
//
// Method: Liu & He, arXiv:1603.01955, Section 3.1: the force-driven periodic
// channel is solved to steady state for many Knudsen numbers (and heights)
// to trace the flow rate Q(Kn) and its Knudsen minimum.  Each channel is
// independent, so one persistent workgroup owns one channel: its populations
// live in LDS for the whole run (144 B per node for the two A-B buffers), the
// workgroup loops over time steps in-kernel and checks convergence itself.
// HBM is touched only to load and store the state.  The per-node arithmetic
// is the same gather (Eqs. 5, 20) and cascaded collision (Eqs. 4, 6-9, 13)
// as the single-channel step, so a channel advances bitwise identically.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "clb.h"
#include "clb_device.hpp"
#include "clb_gather.hpp"
#include "clb_internal.hpp"
#include "clb_trace.hpp"

namespace clb {
namespace {

struct ChanDesc {
  int32_t nx, ny, shift;
  int32_t force;        // 0: no body force; 1: source of Eq. (9); 2: plus its third-order moments
  int64_t off;          // offset (doubles) of the channel's [9][ny][nx] populations
  double r, gx, gy, s3, snu, sq, s8;
};

struct ChanInit {
  int32_t kind, pad;
  double rho0, ux0, uy0, amp;
  uint64_t seed;
};

// Per-channel run state; lives in device memory between calls.
struct ChanState {
  int64_t steps;        // steps taken so far
  double S;             // sum of u_x over the channel at the last check
  double S_prev;        // the check before
  int32_t converged;
  int32_t checks;
};

struct BatchArgs {
  const ChanDesc* ch;
  const int32_t* order;  // workgroup -> channel
  double* state;
  ChanState* cs;
  int64_t max_steps;     // steps allowed in this launch (per channel)
  int32_t check_every;   // convergence check cadence (0: none)
  double tol;            // converged when |S - S_prev| <= tol |S|
};

// Fixed-order block reduction (blockDim.x is a power of two).
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = (int)blockDim.x >> 1; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

template <bool FORCE, bool THIRD>
__device__ void channel_step(const ChanDesc& d, const double* A, double* B, int n) {
  const Gather<0, LdsView> gat{{A, d.nx, d.ny, n}, d.r, 1.0 - d.r, d.shift, 0.0, 0.0};
  const Rates s{d.s3, d.snu, d.sq, d.s8};
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int y = j / d.nx, x = j - y * d.nx;
    double f[9];
    gat(x, y, f);
    collide<FORCE, THIRD>(f, d.gx, d.gy, s);
#pragma unroll
    for (int i = 0; i < 9; ++i) B[i * n + j] = f[i];
  }
}

// One node per thread (n <= blockDim.x): the node, and with it every LDS
// source offset of its gather, stays the same for the whole run, so the
// offsets are worked out once.  a[i]: the population pulled into direction
// i, or its bounce-back part on a wall row; b[k]: the specular part of
// direction 5 + k on a wall row (Eq. 20), x wrapped periodically.  The
// arithmetic per step is that of Gather::operator(), bitwise.
struct NodeSources {
  int a[9], b[4];
  bool bot, top;
};

__device__ __forceinline__ NodeSources node_sources(const ChanDesc& d, int j) {
  const int nx = d.nx, ny = d.ny, n = nx * ny, t = ny - 1;
  const int y = j / nx, x = j - y * nx;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int xsm = d.shift ? xm : x, xsp = d.shift ? xp : x;
  auto at = [&](int i, int xx, int yy) { return i * n + yy * nx + xx; };
  NodeSources q;
  q.bot = y == 0;
  q.top = y == t;
  q.a[0] = at(0, x, y);
  q.a[1] = at(1, xm, y);
  q.a[3] = at(3, xp, y);
  q.a[2] = q.bot ? at(4, x, 0) : at(2, x, y - 1);
  q.a[5] = q.bot ? at(7, x, 0) : at(5, xm, y - 1);
  q.a[6] = q.bot ? at(8, x, 0) : at(6, xp, y - 1);
  q.a[4] = q.top ? at(2, x, t) : at(4, x, y + 1);
  q.a[7] = q.top ? at(5, x, t) : at(7, xp, y + 1);
  q.a[8] = q.top ? at(6, x, t) : at(8, xm, y + 1);
  q.b[0] = q.bot ? at(8, xsm, 0) : q.a[5];
  q.b[1] = q.bot ? at(7, xsp, 0) : q.a[6];
  q.b[2] = q.top ? at(6, xsp, t) : q.a[7];
  q.b[3] = q.top ? at(5, xsm, t) : q.a[8];
  return q;
}

template <bool FORCE, bool THIRD>
__device__ __forceinline__ void node_step(const ChanDesc& d, const NodeSources& q, const double* A, double* B,
                                          int n, int j) {
#pragma clang fp contract(off)
  double f[9], s[4];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = A[q.a[i]];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = A[q.b[k]];
  const double r = d.r, omr = 1.0 - d.r;
  if (q.bot) {
    f[5] = r * f[5] + omr * s[0];
    f[6] = r * f[6] + omr * s[1];
  }
  if (q.top) {
    f[7] = r * f[7] + omr * s[2];
    f[8] = r * f[8] + omr * s[3];
  }
  collide<FORCE, THIRD>(f, d.gx, d.gy, Rates{d.s3, d.snu, d.sq, d.s8});
#pragma unroll
  for (int i = 0; i < 9; ++i) B[i * n + j] = f[i];
}

// Sum over the channel of u_x of the pre-collision state (Eq. 13).
__device__ double channel_sum_ux(const ChanDesc& d, const double* A, int n, double* red) {
  const Gather<0, LdsView> gat{{A, d.nx, d.ny, n}, d.r, 1.0 - d.r, d.shift, 0.0, 0.0};
  double part = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int y = j / d.nx, x = j - y * d.nx;
    double f[9];
    gat(x, y, f);
    double rho, ux, uy;
    rho_u(f, rho, ux, uy);
    part += ux + 0.5 * d.gx;
  }
  return block_sum(part, red);
}

// Persistent batched run: workgroup b advances channel order[b] until it has
// converged or taken max_steps steps in this launch.  Every exit decision is
// uniform across the workgroup (it depends only on LDS-reduced values and
// counters), so all waves leave the loop together.  ONE: every channel has
// at most one node per thread (the launch checks it); the instance then
// carries only the fixed-offset node update, which needs far fewer
// registers than the several-nodes-per-thread loop (no spills in the
// per-step loop).  MAXT: the largest workgroup the instance serves; with at
// most 512 threads the compiler may use up to 256 VGPRs (the batch runs one
// channel per workgroup and few workgroups per CU, so occupancy is not the
// limit, while spills sit in the per-step loop).
template <bool ONE, int MAXT>
__global__ __launch_bounds__(MAXT) void k_batch(BatchArgs a) {
  extern __shared__ double lds[];
  const int c = a.order[blockIdx.x];
  const ChanDesc d = a.ch[c];
  const int n = d.nx * d.ny;
  double* A = lds;
  double* B = lds + 9 * n;
  double* red = lds + 18 * n;
  double* gp = a.state + d.off;
  for (int k = threadIdx.x; k < 9 * n; k += blockDim.x) A[k] = gp[k];
  ChanState st = a.cs[c];
  __syncthreads();
  int64_t taken = 0;
  const bool one = ONE || n <= (int)blockDim.x;   // one node per thread: sources fixed for the run
  const bool mine = (int)threadIdx.x < n;
  NodeSources q{};
  if (one && mine) q = node_sources(d, threadIdx.x);
  // steps to the next convergence check (at multiples of check_every of the
  // channel's step count); a countdown instead of a 64-bit remainder per step
  int64_t to_check = a.check_every > 0 ? a.check_every - st.steps % a.check_every : 0;
  while (!st.converged && taken < a.max_steps) {
    if (one) {
      if (mine) {
        if (d.force == 2)
          node_step<true, true>(d, q, A, B, n, threadIdx.x);
        else if (d.force)
          node_step<true, false>(d, q, A, B, n, threadIdx.x);
        else
          node_step<false, false>(d, q, A, B, n, threadIdx.x);
      }
    } else if (!ONE) {
      if (d.force == 2)
        channel_step<true, true>(d, A, B, n);
      else if (d.force)
        channel_step<true, false>(d, A, B, n);
      else
        channel_step<false, false>(d, A, B, n);
    }
    __syncthreads();
    double* t = A;
    A = B;
    B = t;
    ++taken;
    if (a.check_every > 0 && --to_check == 0) {
      to_check = a.check_every;
      const double S = channel_sum_ux(d, A, n, red);
      st.checks += 1;
      if (fabs(S - st.S) <= a.tol * fabs(S)) st.converged = 1;   // first check: S is NaN
      st.S_prev = st.S;
      st.S = S;
    }
  }
  for (int k = threadIdx.x; k < 9 * n; k += blockDim.x) gp[k] = A[k];
  if (threadIdx.x == 0) {
    st.steps += taken;
    a.cs[c] = st;
  }
}

// Initial state of every channel (same node numbering and generator as the
// single-channel start: node = y * nx + x).
__global__ void k_batch_init(const ChanDesc* ch, const ChanInit* ci, double* state) {
  const ChanDesc d = ch[blockIdx.x];
  const ChanInit c = ci[blockIdx.x];
  const int n = d.nx * d.ny;
  double* gp = state + d.off;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double e[9];
    equilibrium(c.rho0, c.ux0, c.uy0, e);
    if (c.kind == CLB_INIT_PERTURBED) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const uint64_t key = c.seed ^ (9ull * (uint64_t)j + (uint64_t)i);
        const double U = (double)(splitmix64_first(key) >> 11) * (1.0 / 9007199254740992.0);
        e[i] += c.amp * (2.0 * U - 1.0);
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) gp[i * n + j] = e[i];
  }
}

__global__ void k_reset_state(ChanState* cs, int nch) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  ChanState s;
  s.steps = 0;
  s.S = NAN;
  s.S_prev = NAN;
  s.converged = 0;
  s.checks = 0;
  cs[c] = s;
}

// Sum of u_x of the current pre-collision state of each channel (global
// memory, one workgroup of 256 threads per channel).
__global__ __launch_bounds__(256) void k_batch_sum_ux(const ChanDesc* ch, const double* state, double* out) {
  __shared__ double red[256];
  const ChanDesc d = ch[blockIdx.x];
  const int n = d.nx * d.ny;
  out[blockIdx.x] = channel_sum_ux(d, state + d.off, n, red);
}

// Non-finite values among each channel's populations, counted by one
// workgroup of 256 threads per channel (fixed order).
__global__ __launch_bounds__(256) void k_batch_nonfinite(const ChanDesc* ch, const double* state, double* out) {
  __shared__ double red[256];
  const ChanDesc d = ch[blockIdx.x];
  const int n9 = 9 * d.nx * d.ny;
  const double* p = state + d.off;
  double cnt = 0.0;
  for (int k = threadIdx.x; k < n9; k += 256) cnt += (p[k] - p[k] == 0.0) ? 0.0 : 1.0;   // NaN, inf
  const double s = block_sum(cnt, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct BatchLayout {
  size_t state;   // bytes of one state copy
  size_t total;
  int64_t doubles;
};

BatchLayout batch_layout(int32_t nch, const clb_params* ps) {
  BatchLayout L{};
  int64_t tot = 0;
  for (int c = 0; c < nch; ++c) tot += 9 * (int64_t)ps[c].nx * ps[c].ny;
  L.doubles = tot;
  L.state = align256((size_t)tot * sizeof(double));
  L.total = 2 * L.state + align256(nch * sizeof(ChanDesc)) + align256(nch * sizeof(ChanInit)) +
            align256(nch * sizeof(int32_t)) + 2 * align256(nch * sizeof(ChanState)) +
            align256(nch * sizeof(double));
  return L;
}

clb_status err(clb_status st, const char* msg) { return set_error(st, msg); }

#define BATCH_HIP(call)                                                    \
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

struct clb_batch {
  int32_t nch;
  std::vector<clb_params> p;
  std::vector<clb::ChanDesc> desc;      // host copies (kept alive for async uploads)
  std::vector<clb::ChanInit> init;
  std::vector<int32_t> order_natural, order_longest;
  std::vector<double> cost;
  clb::ChanDesc* d_desc;
  clb::ChanInit* d_init;
  int32_t* d_order;
  double* state;
  double* scratch;
  clb::ChanState* cs;
  clb::ChanState* cs_scratch;
  double* sums;
  hipStream_t stream;      // caller's stream: all work runs here
  hipStream_t capture;     // private stream, used only to record the graph
  int32_t threads;
  int32_t longest_first;
  int32_t n_max;
  size_t lds_limit;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int64_t g_max_steps;
  int32_t g_check_every, g_threads, g_longest;
  double g_tol;
  std::vector<clb::ChanState> host_cs;
  std::vector<double> host_sums;
};

namespace {

size_t lds_bytes(const clb_batch* b, int threads) {
  return (18 * (size_t)b->n_max + (size_t)threads) * sizeof(double);
}

clb_status upload_order(clb_batch* b) {
  const std::vector<int32_t>& o = b->longest_first ? b->order_longest : b->order_natural;
  BATCH_HIP(hipMemcpyAsync(b->d_order, o.data(), o.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
  return CLB_OK;
}

clb_status launch_batch(clb_batch* b, hipStream_t st, double* state, clb::ChanState* cs, int64_t max_steps,
                        int32_t check_every, double tol) {
  clb::BatchArgs a{b->d_desc, b->d_order, state, cs, max_steps, check_every, tol};
  const size_t lds = lds_bytes(b, b->threads);
  const bool one = b->n_max <= b->threads;
  if (b->threads <= 512) {
    if (one)
      clb::k_batch<true, 512><<<b->nch, b->threads, lds, st>>>(a);
    else
      clb::k_batch<false, 512><<<b->nch, b->threads, lds, st>>>(a);
  } else {
    if (one)
      clb::k_batch<true, 1024><<<b->nch, b->threads, lds, st>>>(a);
    else
      clb::k_batch<false, 1024><<<b->nch, b->threads, lds, st>>>(a);
  }
  BATCH_HIP(hipGetLastError());
  return CLB_OK;
}

void drop_graph(clb_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

clb_status clb_batch_workspace_size(int32_t nch, const clb_params* params, size_t* bytes) {
  if (!bytes) return clb::err(CLB_EINVAL, "bytes: NULL");
  if (nch < 1 || !params) return clb::err(CLB_EINVAL, "nch/params: need at least one channel");
  for (int c = 0; c < nch; ++c) {
    clb_status st = clb::validate_params(&params[c], nullptr);
    if (st != CLB_OK) return st;
    if (params[c].xbc != CLB_X_PERIODIC) return clb::err(CLB_EINVAL, "xbc: batched channels must be periodic");
    if (params[c].init == CLB_INIT_LINEAR_RHO) return clb::err(CLB_EINVAL, "init: linear start needs pressure mode");
  }
  *bytes = clb::batch_layout(nch, params).total;
  return CLB_OK;
}

clb_status clb_batch_init(int32_t nch, const clb_params* params, void* d_workspace, size_t bytes,
                          void* hip_stream, clb_batch** out) {
  const clb::TraceRange trace("clb_batch_init");
  if (!out) return clb::err(CLB_EINVAL, "out: NULL");
  *out = nullptr;
  size_t need = 0;
  clb_status st = clb_batch_workspace_size(nch, params, &need);
  if (st != CLB_OK) return st;
  if (!d_workspace) return clb::err(CLB_EINVAL, "d_workspace: NULL");
  if (bytes < need) return clb::err(CLB_ENOMEM, "workspace: smaller than clb_batch_workspace_size");
  if ((st = clb::check_device_ptr(d_workspace, need, "d_workspace")) != CLB_OK) return st;

  int dev = 0, lds = 0;
  BATCH_HIP(hipGetDevice(&dev));
  BATCH_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));

  clb_batch* b = new (std::nothrow) clb_batch();
  if (!b) return clb::err(CLB_ENOMEM, "host context allocation failed");
  b->nch = nch;
  b->p.assign(params, params + nch);
  b->lds_limit = (size_t)lds;
  const clb::BatchLayout L = clb::batch_layout(nch, params);
  int64_t off = 0;
  b->n_max = 0;
  for (int c = 0; c < nch; ++c) {
    const clb_params& p = params[c];
    clb_derived d;
    clb::validate_params(&p, &d);
    clb::ChanDesc cd{};
    cd.nx = p.nx;
    cd.ny = p.ny;
    cd.shift = p.cbbsr_shift;
    cd.force = (p.gx != 0.0 || p.gy != 0.0) ? (p.forcing ? 2 : 1) : 0;
    cd.off = off;
    cd.r = d.r;
    cd.gx = p.gx;
    cd.gy = p.gy;
    cd.s3 = p.s3;
    cd.snu = d.s_nu;
    cd.sq = d.s_q;
    cd.s8 = p.s8;
    b->desc.push_back(cd);
    clb::ChanInit ci{};
    ci.kind = p.init;
    ci.rho0 = p.rho0;
    ci.ux0 = p.ux0;
    ci.uy0 = p.uy0;
    ci.amp = p.init == CLB_INIT_PERTURBED ? p.init_amp : 0.0;
    ci.seed = p.seed;
    b->init.push_back(ci);
    off += 9 * (int64_t)p.nx * p.ny;
    b->n_max = std::max(b->n_max, p.nx * p.ny);
    // steps to steady state scale like H^2 / nu with nu = tau_tilde / 3 (Eqs. 14, 18)
    b->cost.push_back((double)p.nx * p.ny * (double)p.ny * p.ny / d.tau_tilde);
  }
  if (lds_bytes(b, 64) > b->lds_limit) {
    delete b;
    return clb::err(CLB_EINVAL, "nx*ny: largest channel does not fit in one workgroup's LDS");
  }
  b->order_natural.resize(nch);
  std::iota(b->order_natural.begin(), b->order_natural.end(), 0);
  b->order_longest = b->order_natural;
  std::stable_sort(b->order_longest.begin(), b->order_longest.end(),
                   [b](int x, int y) { return b->cost[x] > b->cost[y]; });

  char* q = static_cast<char*>(d_workspace);
  b->state = reinterpret_cast<double*>(q);
  q += L.state;
  b->scratch = reinterpret_cast<double*>(q);
  q += L.state;
  b->d_desc = reinterpret_cast<clb::ChanDesc*>(q);
  q += clb::align256(nch * sizeof(clb::ChanDesc));
  b->d_init = reinterpret_cast<clb::ChanInit*>(q);
  q += clb::align256(nch * sizeof(clb::ChanInit));
  b->d_order = reinterpret_cast<int32_t*>(q);
  q += clb::align256(nch * sizeof(int32_t));
  b->cs = reinterpret_cast<clb::ChanState*>(q);
  q += clb::align256(nch * sizeof(clb::ChanState));
  b->cs_scratch = reinterpret_cast<clb::ChanState*>(q);
  q += clb::align256(nch * sizeof(clb::ChanState));
  b->sums = reinterpret_cast<double*>(q);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->threads = 1;
  while (b->threads < b->n_max && b->threads < 1024) b->threads <<= 1;
  b->threads = std::max(b->threads, 64);
  while (b->threads > 64 && lds_bytes(b, b->threads) > b->lds_limit) b->threads >>= 1;
  b->longest_first = 1;
  b->host_cs.resize(nch);
  b->host_sums.resize(nch);

  auto fail_init = [b](hipError_t e, const char* where) {
    char m[256];
    snprintf(m, sizeof(m), "%s: %s", where, hipGetErrorString(e));
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return clb::set_error(CLB_EHIP, m);
  };
  hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e != hipSuccess) return fail_init(e, "hipStreamCreateWithFlags");
  for (const void* k : {reinterpret_cast<const void*>(&clb::k_batch<true, 512>),
                        reinterpret_cast<const void*>(&clb::k_batch<false, 512>),
                        reinterpret_cast<const void*>(&clb::k_batch<true, 1024>),
                        reinterpret_cast<const void*>(&clb::k_batch<false, 1024>)}) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(b, 1024));
    if (e != hipSuccess) break;
  }
  if (e != hipSuccess) (void)hipGetLastError();   // not needed on every runtime
  e = hipMemcpyAsync(b->d_desc, b->desc.data(), nch * sizeof(clb::ChanDesc), hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return fail_init(e, "upload channel table");
  e = hipMemcpyAsync(b->d_init, b->init.data(), nch * sizeof(clb::ChanInit), hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return fail_init(e, "upload channel starts");
  clb::k_batch_init<<<nch, 256, 0, b->stream>>>(b->d_desc, b->d_init, b->state);
  clb::k_reset_state<<<(nch + 255) / 256, 256, 0, b->stream>>>(b->cs, nch);
  e = hipGetLastError();
  if (e != hipSuccess) return fail_init(e, "batch init kernels");
  if (upload_order(b) != CLB_OK) {
    (void)hipStreamDestroy(b->capture);
    delete b;
    return CLB_EHIP;
  }
  // The uploads read host vectors owned by b; finish them before returning.
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail_init(e, "hipStreamSynchronize");
  *out = b;
  return CLB_OK;
}

clb_status clb_batch_set_launch(clb_batch* b, int32_t threads, int32_t longest_first) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
    return clb::err(CLB_EINVAL, "threads: must be 64, 128, 256, 512 or 1024");
  if (longest_first != 0 && longest_first != 1) return clb::err(CLB_EINVAL, "longest_first: must be 0 or 1");
  if (lds_bytes(b, threads) > b->lds_limit) return clb::err(CLB_EINVAL, "threads: LDS budget exceeded");
  const bool reorder = longest_first != b->longest_first;
  b->threads = threads;
  b->longest_first = longest_first;
  if (reorder) {
    clb_status st = upload_order(b);
    if (st != CLB_OK) return st;
    BATCH_HIP(hipStreamSynchronize(b->stream));
  }
  return CLB_OK;
}

clb_status clb_batch_tune(clb_batch* b, int32_t probe_steps, int32_t* h_threads, int32_t* h_longest_first) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (probe_steps < 1) return clb::err(CLB_EINVAL, "probe_steps: must be >= 1");
  hipEvent_t e0, e1;
  BATCH_HIP(hipEventCreate(&e0));
  BATCH_HIP(hipEventCreate(&e1));
  float best = 0.0f;
  int32_t best_t = b->threads, best_o = b->longest_first;
  const int32_t keep_t = b->threads, keep_o = b->longest_first;
  clb_status st = CLB_OK;
  for (int o = 1; o >= 0 && st == CLB_OK; --o) {
    for (int t = 64; t <= 1024 && st == CLB_OK; t <<= 1) {
      if (lds_bytes(b, t) > b->lds_limit) continue;
      if (t > 2 * std::max(64, b->n_max)) continue;
      if ((st = clb_batch_set_launch(b, t, o)) != CLB_OK) break;
      // Probe on a copy of the state: the batch itself does not advance.
      hipError_t e = hipMemcpyAsync(b->scratch, b->state, (size_t)clb::batch_layout(b->nch, b->p.data()).doubles *
                                    sizeof(double), hipMemcpyDeviceToDevice, b->stream);
      if (e != hipSuccess) { st = clb::set_error(CLB_EHIP, hipGetErrorString(e)); break; }
      clb::k_reset_state<<<(b->nch + 255) / 256, 256, 0, b->stream>>>(b->cs_scratch, b->nch);
      (void)hipEventRecord(e0, b->stream);
      if ((st = launch_batch(b, b->stream, b->scratch, b->cs_scratch, probe_steps, 0, 0.0)) != CLB_OK) break;
      (void)hipEventRecord(e1, b->stream);
      e = hipEventSynchronize(e1);
      if (e != hipSuccess) { st = clb::set_error(CLB_EHIP, hipGetErrorString(e)); break; }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best == 0.0f || ms < best) {
        best = ms;
        best_t = t;
        best_o = o;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != CLB_OK) {
    clb_batch_set_launch(b, keep_t, keep_o);
    return st;
  }
  if ((st = clb_batch_set_launch(b, best_t, best_o)) != CLB_OK) return st;
  if (h_threads) *h_threads = best_t;
  if (h_longest_first) *h_longest_first = best_o;
  return CLB_OK;
}

clb_status clb_batch_run(clb_batch* b, int64_t max_steps, int32_t check_every, double tol, int64_t* h_steps,
                         int32_t* h_converged) {
  const clb::TraceRange trace("clb_batch_run");
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (max_steps < 0) return clb::err(CLB_EINVAL, "max_steps: must be >= 0");
  if (check_every < 0) return clb::err(CLB_EINVAL, "check_every: must be >= 0");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return clb::err(CLB_EINVAL, "tol: must be finite and >= 0");
  // The launch is recorded once into a graph and replayed while the run
  // arguments and launch shape stay the same.
  if (!b->exec || b->g_max_steps != max_steps || b->g_check_every != check_every || b->g_tol != tol ||
      b->g_threads != b->threads || b->g_longest != b->longest_first) {
    drop_graph(b);
    BATCH_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    clb_status st = launch_batch(b, b->capture, b->state, b->cs, max_steps, check_every, tol);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture, &g);
    if (st != CLB_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return clb::set_error(CLB_EHIP, hipGetErrorString(e));
    b->graph = g;
    BATCH_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_max_steps = max_steps;
    b->g_check_every = check_every;
    b->g_tol = tol;
    b->g_threads = b->threads;
    b->g_longest = b->longest_first;
  }
  BATCH_HIP(hipGraphLaunch(b->exec, b->stream));
  if (h_steps || h_converged) {
    BATCH_HIP(hipMemcpyAsync(b->host_cs.data(), b->cs, b->nch * sizeof(clb::ChanState), hipMemcpyDeviceToHost,
                             b->stream));
    BATCH_HIP(hipStreamSynchronize(b->stream));
    for (int c = 0; c < b->nch; ++c) {
      if (h_steps) h_steps[c] = b->host_cs[c].steps;
      if (h_converged) h_converged[c] = b->host_cs[c].converged;
    }
  }
  return CLB_OK;
}

clb_status clb_batch_flow_rate(clb_batch* b, double* h_Q) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (!h_Q) return clb::err(CLB_EINVAL, "h_Q: NULL");
  for (int c = 0; c < b->nch; ++c)
    if (b->p[c].gx == 0.0) return clb::err(CLB_ESTATE, "clb_batch_flow_rate: every channel needs gx != 0");
  clb::k_batch_sum_ux<<<b->nch, 256, 0, b->stream>>>(b->d_desc, b->state, b->sums);
  BATCH_HIP(hipGetLastError());
  BATCH_HIP(hipMemcpyAsync(b->host_sums.data(), b->sums, b->nch * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BATCH_HIP(hipStreamSynchronize(b->stream));
  for (int c = 0; c < b->nch; ++c) {
    const clb_params& p = b->p[c];
    const double H = (double)p.ny;
    // Section 3.1: Q = (int u_x dy) / (F_x H^2 sqrt(RT/2) / p), per column
    h_Q[c] = (b->host_sums[c] / p.nx) * std::sqrt(6.0) / (3.0 * p.gx * H * H);
  }
  return CLB_OK;
}

clb_status clb_batch_check_finite(clb_batch* b, int32_t* h_ok) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (!h_ok) return clb::err(CLB_EINVAL, "h_ok: NULL");
  clb::k_batch_nonfinite<<<b->nch, 256, 0, b->stream>>>(b->d_desc, b->state, b->sums);
  BATCH_HIP(hipGetLastError());
  BATCH_HIP(hipMemcpyAsync(b->host_sums.data(), b->sums, b->nch * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BATCH_HIP(hipStreamSynchronize(b->stream));
  int bad = 0;
  for (int c = 0; c < b->nch; ++c) {
    h_ok[c] = b->host_sums[c] == 0.0 ? 1 : 0;
    bad += !h_ok[c];
  }
  if (bad) return clb::err(CLB_EUNSTABLE, "populations: non-finite values in at least one channel");
  return CLB_OK;
}

clb_status clb_batch_get_populations(clb_batch* b, int32_t ch, double* d_out) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (ch < 0 || ch >= b->nch) return clb::err(CLB_EINVAL, "ch: out of range");
  const size_t bytes = 9 * (size_t)b->p[ch].nx * b->p[ch].ny * sizeof(double);
  clb_status st = clb::check_device_ptr(d_out, bytes, "d_out");
  if (st != CLB_OK) return st;
  BATCH_HIP(hipMemcpyAsync(d_out, b->state + b->desc[ch].off, bytes, hipMemcpyDeviceToDevice, b->stream));
  return CLB_OK;
}

clb_status clb_batch_set_populations(clb_batch* b, int32_t ch, const double* d_in) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  if (ch < 0 || ch >= b->nch) return clb::err(CLB_EINVAL, "ch: out of range");
  const size_t bytes = 9 * (size_t)b->p[ch].nx * b->p[ch].ny * sizeof(double);
  clb_status st = clb::check_device_ptr(d_in, bytes, "d_in");
  if (st != CLB_OK) return st;
  BATCH_HIP(hipMemcpyAsync(b->state + b->desc[ch].off, d_in, bytes, hipMemcpyDeviceToDevice, b->stream));
  return CLB_OK;
}

clb_status clb_batch_reset(clb_batch* b) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  clb::k_reset_state<<<(b->nch + 255) / 256, 256, 0, b->stream>>>(b->cs, b->nch);
  BATCH_HIP(hipGetLastError());
  return CLB_OK;
}

clb_status clb_batch_destroy(clb_batch* b) {
  if (!b) return clb::err(CLB_EINVAL, "batch: NULL");
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
  return CLB_OK;
}

}  // extern "C"
