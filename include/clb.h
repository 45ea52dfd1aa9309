/*
 * clb.h -- C ABI of the MI355X (gfx950) cascaded lattice Boltzmann library.
 *
 * Method: Liu & He, "Numerical modelling of microchannel gas flows in the
 * transition flow regime using the cascaded lattice Boltzmann method",
 * arXiv:1603.01955.  D2Q9 cascaded collision with semi-implicit forcing
 * (Section 2.1, Eqs. 1-14), Bosanquet-type effective viscosity setting the
 * shear rate from Kn (Section 2.2, Eqs. 15-18), combined bounce-back /
 * specular-reflection walls matched to a modified second-order slip law
 * (Section 2.3, Eqs. 19-21), periodic or pressure inlet/outlet (Section 3).
 *
 * Conventions shared by every entry point
 *  - Lattice units: dx = dt = c = 1, c_s^2 = 1/3, p = rho/3.
 *  - Grid: nx x ny fluid nodes; row y sits at height y + 1/2 between walls
 *    placed half a spacing below row 0 and above row ny-1, so the channel
 *    height is H = ny (the N of Eq. 18).  Column x sits at x + 1/2; in
 *    pressure mode the inlet plane is x = 0 and the outlet plane x = nx.
 *  - Populations: FP64, structure of arrays, P[i][y][x] with x fastest,
 *    direction i ordered as in Eq. (1): (0,0) (1,0) (0,1) (-1,0) (0,-1)
 *    (1,1) (-1,1) (-1,-1) (1,-1).  The stored state is the post-collision
 *    transformed population of Eq. (4); one step is streaming (Eq. 5) with
 *    the boundaries, then the collision.
 *  - Memory: the caller owns all device memory and the stream.  The library
 *    allocates only a small host-side context and never calls hipMalloc.
 *    "d_" pointers are device pointers, "h_" pointers host pointers.
 *  - Asynchrony: every call enqueues work on the context's stream and
 *    returns; only calls that write a host pointer synchronise that stream.
 *  - Errors: every call returns a clb_status; CLB_OK is 0.  The message of
 *    the last failure on the calling thread is returned by clb_last_error().
 *    Invalid arguments are rejected before any device work is enqueued.
 */
#ifndef CLB_H
#define CLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden symbol visibility; the declarations of
 * this header are its exported interface. */
#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

typedef enum clb_status {
  CLB_OK = 0,
  CLB_EINVAL = -1,     /* invalid argument; the message names the field      */
  CLB_ENOMEM = -2,     /* caller's workspace smaller than required            */
  CLB_EHIP = -3,       /* a HIP runtime call failed; message has its text     */
  CLB_ESTATE = -4,     /* call not valid for this context (e.g. wrong mode)   */
  CLB_EUNSTABLE = -5   /* non-finite populations detected                     */
} clb_status;

typedef enum clb_xbc {
  CLB_X_PERIODIC = 0,  /* periodic inlet/outlet, body-force driven (Section 3.1) */
  CLB_X_PRESSURE = 1   /* pressure inlet/outlet, local Kn(x) (Section 3.2)       */
} clb_xbc;

typedef enum clb_init_kind {
  CLB_INIT_UNIFORM = 0,    /* f = f^eq(rho0, (ux0, uy0)) everywhere (Eq. 11)        */
  CLB_INIT_LINEAR_RHO = 1, /* f = f^eq(rho(x), 0), rho linear from p_ratio*rho_out
                              at x = 0 to rho_out at x = nx                        */
  CLB_INIT_PERTURBED = 2   /* f_i = f_i^eq(rho0, u0) + init_amp * (2U - 1) with U the
                              top 53 bits of SplitMix64 (Steele, Lea & Flood 2014)
                              of key = seed XOR (9 * (y*nx + x) + i), times 2^-53   */
} clb_init_kind;

/* Problem statement.  clb_params_default() fills the values of Section 3:
 * a = 2, sigma = 1, B2 = 0.55, s3 = 1.1, s8 = 1.2. */
typedef struct clb_params {
  int32_t nx, ny;        /* fluid nodes along / across the channel (>= 1; pressure: nx >= 2) */
  int32_t xbc;           /* clb_xbc                                                        */
  int32_t init;          /* clb_init_kind                                                  */
  double kn;             /* Kn (periodic) or outlet Kn_out (pressure), > 0    Eqs. 18, Sec. 3.2 */
  double a;              /* Bosanquet rarefaction factor, >= 0                Eq. 16          */
  double sigma;          /* TMAC in (0, 2]; A1 = (1 - 0.1817 sigma)(2 - sigma)/sigma  Eq. 19, Sec. 3 */
  double A1;             /* first-order slip coefficient B1*sigma_v; NaN -> from sigma         */
  double A2;             /* second-order slip coefficient B2, >= 0            Eq. 19, 21      */
  double r;              /* bounce-back fraction in [0, 1]; NaN -> Eq. 21 from A1              */
  double s3, s8;         /* bulk and fourth-order relaxation rates in (0, 2)  Eq. 14, Sec. 3  */
  double gx, gy;         /* body acceleration F (periodic mode only; 0 in pressure mode) Eq. 9 */
  double p_ratio;        /* p_in / p_out (pressure mode), > 0                 Sec. 3.2        */
  double rho_out;        /* outlet density (pressure mode), > 0                               */
  double rho0, ux0, uy0; /* uniform start (CLB_INIT_UNIFORM / PERTURBED)                       */
  double init_amp;       /* perturbation amplitude (CLB_INIT_PERTURBED), >= 0                  */
  uint64_t seed;         /* perturbation seed                                                  */
  double tq_den;         /* denominator of Eq. 21 (16 as printed; 24 = exact-slip variant)     */
  int32_t cbbsr_shift;   /* Eq. 20 specular source: 1 = neighbour x-1 / x+1 (default),
                            0 = the same node                                                   */
  int32_t forcing;       /* body-force source: 0 = Eq. 9 as printed (default); 1 = Eq. 9 plus the
                            third-order moments (1 - s_q/2) rho F / 3 of a second-order (Guo-type)
                            force term in k_xxy (F_y) and k_xyy (F_x), with which Eq. 21's
                            denominator 16 gives the slip law of Eq. 19 exactly.  No effect
                            without a force (pressure mode).                                    */
} clb_params;

/* Derived constants (host-only).  In pressure mode s_nu, s_q and tau_tilde
 * are the outlet values; inside the step they are evaluated per column. */
typedef struct clb_derived {
  double A1;             /* B1 * sigma_v actually used                       */
  double r;              /* bounce-back fraction, Eq. 21                     */
  double tau_tilde;      /* s_nu^-1 - 1/2 = sqrt(6/pi) N Kn / (1 + a Kn), Eq. 18 */
  double s_nu;           /* shear rate s4 = s5, Eq. 18                       */
  double s_q;            /* third-order rate s6 = s7, Eq. 21                 */
} clb_derived;

typedef struct clb_ctx clb_ctx;

/* Fill *p with the Section 3 defaults and a 1 x 1 periodic grid. */
void clb_params_default(clb_params* p);

/* Validate *p and compute the derived constants (Eqs. 18, 21).  Host only,
 * no device needed.  CLB_EINVAL if *p is out of range. */
clb_status clb_derive(const clb_params* p, clb_derived* out);

/* Device workspace in bytes needed by clb_init for *p: two population buffers
 * (72 bytes per node; rows are padded to whole segments of L lanes,
 * L = min(1024, next power of two >= nx)) plus small per-column and per-row
 * scratch (diagnostics, local relaxation rates, ghost columns).
 * The device-side layout of a buffer is internal; populations cross the ABI
 * only in the [9][ny][nx] layout (clb_get_populations / clb_set_populations). */
clb_status clb_workspace_size(const clb_params* p, size_t* bytes);

/* Create a context over the caller's workspace (device memory of at least
 * clb_workspace_size bytes, 8-byte aligned, owned by the caller and kept alive
 * until clb_destroy) and enqueue the initial state (init kind of *p) on
 * hip_stream (a hipStream_t; NULL means the null stream).  The context keeps
 * its own copy of *p. */
clb_status clb_init(const clb_params* p, void* d_workspace, size_t bytes,
                    void* hip_stream, clb_ctx** out);

/* Advance nsteps >= 0 time steps (stream + boundaries + collision, Eqs. 4-5,
 * 20).  Asynchronous, unless checks are switched on (clb_set_check_every):
 * then CLB_EUNSTABLE reports non-finite populations at a check. */
clb_status clb_step(clb_ctx* c, int64_t nsteps);

/* Number of steps taken since clb_init / the last clb_set_populations. */
clb_status clb_steps_done(const clb_ctx* c, int64_t* h_steps);

/* Macroscopic fields of the current pre-collision state (the populations
 * after streaming and boundaries at the current time level), Eqs. 12-13:
 * rho = sum f, rho u = sum e f + rho F/2.  Each output is a device array of
 * ny * nx doubles, [y][x]; any of them may be NULL. */
clb_status clb_moments(clb_ctx* c, double* d_rho, double* d_ux, double* d_uy);

/* Per-column sums of the pre-collision state: d_m[x] = sum_y rho u_x (the
 * mass flow m of Section 3.2), d_su[x] = sum_y u_x, d_rhoc[x] = centre-line
 * density (middle row, or mean of the two middle rows for even ny).  Device
 * arrays of nx doubles; any may be NULL.  Fixed summation order. */
clb_status clb_column_sums(clb_ctx* c, double* d_m, double* d_su, double* d_rhoc);

/* Mass flow (Section 3.2): optional per-column d_m_col[nx] (device) and the
 * column mean written to *h_m_mean (host; synchronises the stream; may be NULL,
 * then nothing is synchronised). */
clb_status clb_massflow(clb_ctx* c, double* d_m_col, double* h_m_mean);

/* Dimensionless flow rate of Section 3.1, Q = (int u_x dy)/(F_x H^2 sqrt(RT/2)/p)
 * with F_x = rho0 gx, RT = 1/3, p = rho0/3, the integral a midpoint sum over
 * rows, averaged over columns.  Periodic mode with gx != 0 only.  Synchronises. */
clb_status clb_flow_rate(clb_ctx* c, double* h_Q);

/* Pressure deviation along the centre line (Section 3.2):
 * d_dp[x] = (p_c(x) - p_l(x)) / p_out with p_l falling linearly from p_in at
 * x = 0 to p_out at x = nx; optional d_rho_c[x].  Pressure mode only. */
clb_status clb_pressure_deviation(clb_ctx* c, double* d_dp, double* d_rho_c);

/* Copy the current post-collision populations out / in, [9][ny][nx] doubles
 * in device memory.  clb_set_populations resets the step counter. */
clb_status clb_get_populations(clb_ctx* c, double* d_out);
clb_status clb_set_populations(clb_ctx* c, const double* d_in);

/* Failure detection: *h_ok = 1 if every population is finite, else 0 and the
 * call returns CLB_EUNSTABLE.  Synchronises. */
clb_status clb_check_finite(clb_ctx* c, int32_t* h_ok);

/* Failure detection inside clb_step (the paper has none; an auxiliary check
 * for long runs): with check_every > 0, clb_step stops at every step count
 * that is a multiple of check_every (counted since clb_init or the last
 * clb_set_populations), counts the non-finite populations of the state, and
 * returns CLB_EUNSTABLE at the first check that finds any, leaving the
 * state and the step counter at that step (steps after it are not taken).
 * Each check synchronises the stream; between checks clb_step stays
 * asynchronous.  0 (default) switches the checks off.  CLB_EINVAL if
 * check_every < 0. */
clb_status clb_set_check_every(clb_ctx* c, int64_t check_every);

/* Step-kernel launch shape (tuning; defaults are chosen by measurement):
 * block_x threads per row segment (64, 128, 256, 512 or 1024) and
 * xcd_remap = 1 to map consecutive row segments onto the same XCD. */
clb_status clb_set_launch(clb_ctx* c, int32_t block_x, int32_t xcd_remap);

/* Temporal blocking (tuning): steps = k in 2..4 advances k steps per launch
 * -- each workgroup computes the first step for its tile and a (k - 1)-node
 * halo into LDS, the next ones from LDS on a region one node smaller each
 * time, and writes only the last.  Periodic mode (nx >= 64; narrower grids
 * step one at a time): 64-column tiles, a node update moves about 144 / k
 * bytes plus the halo reads (k = 3, the default: about 59 bytes).  Pressure
 * mode (channels of at most 48 rows on the column-kernel path; others step
 * one at a time): tiles of whole columns, the edge workgroups rebuilding the
 * ghost columns from the LDS values of each step; default k = 4.  A shorter
 * remainder of clb_step takes fewer.  steps = 1: one step per launch.  All
 * give bitwise the same populations.  CLB_EINVAL for other values. */
clb_status clb_set_steps_per_launch(clb_ctx* c, int32_t steps);

/* Pressure-mode kernel choice (tuning; Section 3.2 step): 0 = by grid size
 * (default), 1 = column kernel (each workgroup owns whole columns and takes
 * the local Kn from its own centre rows; best for the small channels of the
 * paper), 2 = row kernel (a prep launch computes the per-column rates and
 * ghost columns, then the step streams whole row segments; best for large
 * grids).  Both give bitwise the same populations.  CLB_EINVAL for other
 * values; no effect in periodic mode. */
clb_status clb_set_pressure_path(clb_ctx* c, int32_t path);

/* Launch-overhead control for small grids: with steps_per_graph > 0,
 * clb_step replays a hipGraph of steps_per_graph recorded step launches
 * (recorded on first use, on a private stream, and replayed on the context's
 * stream) and launches any remainder one by one.  0 (default) disables it.
 * Results are identical either way. */
clb_status clb_set_graph_steps(clb_ctx* c, int32_t steps_per_graph);

/* Release the host context (not the caller's workspace or stream). */
clb_status clb_destroy(clb_ctx* c);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the mass
 * flow of clb_massflow computed from populations the caller holds, with no
 * context and no workspace.  d_P holds post-collision populations in the
 * [9][ny][nx] layout of clb_get_populations (device memory, read only) of
 * the problem *p; the outputs are those of clb_massflow: per-column
 * d_m_col[nx] (device, may be NULL) and the column mean *h_m_mean (host, may
 * be NULL; synchronises hip_stream).  Work is enqueued on hip_stream.  The
 * scratch (the per-column sums when d_m_col is NULL, and the mean) is a fixed
 * device array of the library, CLB_NOALLOC_MAX_NX + 32 doubles per GPU, held
 * until the process ends; the call never allocates device memory.  Calls
 * that overlap on one GPU share that array and race.  CLB_EINVAL for an
 * invalid *p, nx > CLB_NOALLOC_MAX_NX, or pointers that are not device
 * memory of the needed size. */
#define CLB_NOALLOC_MAX_NX (1 << 20)
clb_status clb_massflow_noalloc(const clb_params* p, const double* d_P, double* d_m_col, double* h_m_mean,
                                void* hip_stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent small periodic channels advanced by one
 * persistent launch (the Kn sweep of Section 3.1 that traces the flow rate
 * Q(Kn) and its Knudsen minimum).  Channel c is described by params[c]
 * (periodic, uniform or perturbed start); its two population buffers must fit
 * in one workgroup's LDS (144 * nx * ny bytes plus a reduction area, e.g.
 * nx * ny <= 1024 on MI355X).  Each channel advances exactly as a
 * single-channel context with the same parameters would.
 * ------------------------------------------------------------------------- */
typedef struct clb_batch clb_batch;

/* Device workspace in bytes for a batch of nch channels. */
clb_status clb_batch_workspace_size(int32_t nch, const clb_params* params, size_t* bytes);

/* Create a batch over the caller's workspace and enqueue every channel's
 * start; params is copied.  Synchronises hip_stream once (table uploads). */
clb_status clb_batch_init(int32_t nch, const clb_params* params, void* d_workspace, size_t bytes,
                          void* hip_stream, clb_batch** out);

/* Advance every channel that has not converged by up to max_steps steps in
 * one persistent launch (recorded once as a hipGraph and replayed while the
 * arguments stay the same).  With check_every > 0, every check_every steps
 * (counted from the channel's start) the channel computes S = sum over its
 * nodes of u_x of the pre-collision state and stops once
 * |S - S_previous| <= tol * |S|.  h_steps[nch] (total steps per channel) and
 * h_converged[nch] are written if non-NULL, which synchronises the stream. */
clb_status clb_batch_run(clb_batch* b, int64_t max_steps, int32_t check_every, double tol,
                         int64_t* h_steps, int32_t* h_converged);

/* Dimensionless flow rate Q of every channel (Section 3.1, as clb_flow_rate),
 * h_Q[nch] on the host; every channel needs gx != 0.  Synchronises. */
clb_status clb_batch_flow_rate(clb_batch* b, double* h_Q);

/* Launch shape: threads per workgroup (64, 128, 256, 512 or 1024) and the
 * channel-to-workgroup order (1: estimated longest run first, 0: as given). */
clb_status clb_batch_set_launch(clb_batch* b, int32_t threads, int32_t longest_first);

/* Autotuner: time every admissible launch shape for probe_steps steps on a
 * scratch copy of the state (the batch does not advance), keep the fastest
 * and report it.  Synchronises. */
clb_status clb_batch_tune(clb_batch* b, int32_t probe_steps, int32_t* h_threads, int32_t* h_longest_first);

/* Copy channel ch's post-collision populations out / in ([9][ny][nx], device). */
clb_status clb_batch_get_populations(clb_batch* b, int32_t ch, double* d_out);
clb_status clb_batch_set_populations(clb_batch* b, int32_t ch, const double* d_in);

/* Forget step counts and convergence history (the populations are kept). */
clb_status clb_batch_reset(clb_batch* b);

/* Failure detection: h_ok[nch] = 1 where every population of the channel is
 * finite, else 0; CLB_EUNSTABLE if any channel is not.  Synchronises. */
clb_status clb_batch_check_finite(clb_batch* b, int32_t* h_ok);

/* Release the host context (synchronises the stream first). */
clb_status clb_batch_destroy(clb_batch* b);

/* ---------------------------------------------------------------------------
 * Batch of pressure-driven long channels (Section 3.2, the mass-flow study:
 * dimensionless mass flow S = m / m_ns against Kn_out, or against
 * Kn_ave = (Kn_in + Kn_out) / 2, at a fixed pressure ratio and TMAC).
 * Channel c is described by params[c]: every channel is in pressure mode and
 * all share nx, ny and cbbsr_shift; Kn_out (kn), p_ratio, rho_out, a, sigma
 * or A1, A2, r, s3, s8, tq_den and the start may differ.  One launch per step
 * advances every channel that is still running; each channel advances
 * bitwise as a single-channel context with the same parameters would.
 * Populations stay in the caller's workspace (device layout, two buffers
 * per channel, 144 * nx * ny bytes per channel plus padding).
 * ------------------------------------------------------------------------- */
typedef struct clb_pbatch clb_pbatch;

/* Device workspace in bytes for nch channels; CLB_EINVAL names the first
 * field that is invalid or differs between channels. */
clb_status clb_pbatch_workspace_size(int32_t nch, const clb_params* params, size_t* bytes);

/* Create the batch over the caller's workspace and enqueue every channel's
 * start; params is copied.  Synchronises hip_stream once (table upload). */
clb_status clb_pbatch_init(int32_t nch, const clb_params* params, void* d_workspace, size_t bytes,
                           void* hip_stream, clb_pbatch** out);

/* Advance every running channel by nsteps steps (asynchronous). */
clb_status clb_pbatch_step(clb_pbatch* b, int64_t nsteps);

/* Advance the running channels by up to max_steps steps.  With
 * check_every > 0 (at most 100000), after every check_every steps of this
 * call each running channel compares its column-mean mass flow
 * m = (1/nx) sum_x sum_y rho u_x (pre-collision state) with its value at the
 * previous check and stops once |m - m_previous| <= tol * |m|; the chunk of
 * steps and its check are recorded once as a hipGraph and replayed, and the
 * call returns early when every channel has stopped.  Synchronises once per
 * chunk.  h_steps[nch] (steps per channel) and h_converged[nch] are written
 * if non-NULL. */
clb_status clb_pbatch_run(clb_pbatch* b, int64_t max_steps, int32_t check_every, double tol,
                          int64_t* h_steps, int32_t* h_converged);

/* Steps per launch (tuning): k = 2..4 (default 4) advances the running
 * channels k steps per launch (the steps before the last kept in LDS, as
 * clb_set_steps_per_launch in pressure mode) where the grid allows it
 * (ny <= 48, column kernel), 1 one step per launch.  Bitwise the same
 * populations.  CLB_EINVAL otherwise. */
clb_status clb_pbatch_set_steps_per_launch(clb_pbatch* b, int32_t steps);

/* Kernel choice (tuning): 0 = by total size (default; the row form from
 * 2^21 nodes over all channels), 1 = column kernel (each workgroup owns whole
 * columns of one channel), 2 = row kernel (a prep launch computes every
 * running channel's per-column rates and ghost columns, then one launch
 * streams whole row segments of all channels).  Both give bitwise the same
 * populations.  CLB_EINVAL for other values. */
clb_status clb_pbatch_set_path(clb_pbatch* b, int32_t path);

/* Host arrays of nch values, either may be NULL (not both): h_m the
 * column-mean mass flow of each channel's current state (as in
 * clb_pbatch_run; synchronises), h_m_ns the continuum no-slip mass flow of a
 * long channel with the same pressures and gas (isothermal lubrication
 * limit, m_ns = H^3 (p_in^2 - p_out^2) / (24 mu RT L) with RT = 1/3,
 * p = rho/3, H = ny, L = nx, mu = (1/3) sqrt(6/pi) rho_out Kn_out H from
 * Eqs. 15-17 without the Bosanquet factor).  S = h_m / h_m_ns. */
clb_status clb_pbatch_massflow(clb_pbatch* b, double* h_m, double* h_m_ns);

/* Per-column sums of channel ch, as clb_column_sums (device arrays [nx],
 * each may be NULL). */
clb_status clb_pbatch_column_sums(clb_pbatch* b, int32_t ch, double* d_m, double* d_su, double* d_rhoc);

/* Centre-line pressure deviation of channel ch, as clb_pressure_deviation
 * (device array [nx]). */
clb_status clb_pbatch_pressure_deviation(clb_pbatch* b, int32_t ch, double* d_dp);

/* Copy channel ch's post-collision populations out / in ([9][ny][nx],
 * device).  Setting them leaves the channel's step count and run state
 * as they are. */
clb_status clb_pbatch_get_populations(clb_pbatch* b, int32_t ch, double* d_out);
clb_status clb_pbatch_set_populations(clb_pbatch* b, int32_t ch, const double* d_in);

/* Failure detection: h_ok[nch] = 1 where every population of the channel is
 * finite, else 0; the call returns CLB_EUNSTABLE if any channel is not.
 * Synchronises. */
clb_status clb_pbatch_check_finite(clb_pbatch* b, int32_t* h_ok);

/* Release the host context (synchronises the stream first). */
clb_status clb_pbatch_destroy(clb_pbatch* b);

/* ---------------------------------------------------------------------------
 * Differentiation: hand-written adjoint of the pressure-driven run (Section
 * 3.2).  A run is T steps from the start of *p (normally the linear-density
 * start, CLB_INIT_LINEAR_RHO); its loss is
 *   L = (1/nx) sum_x (dp(x) - dp*(x))^2 + ((m - m*) / m*)^2
 * with dp the centre-line pressure deviation (as clb_pressure_deviation) and
 * m = sum_y rho u_x at the outlet column x = nx - 1, both of the state after T
 * steps.  Gradients are taken with respect to the Bosanquet factor a
 * (Eq. 16, through Eq. 18 and the local Kn), the second-order slip
 * coefficient A2 = B2 (Eq. 21), the bounce-back fraction r (Eq. 20), and A1
 * (Eq. 21, which enters only through r).  The forward run keeps ceil(T/K)
 * checkpoints; the backward sweep recomputes each K-step segment from its
 * checkpoint (K ~ sqrt(T) balances memory and recompute).
 * ------------------------------------------------------------------------- */
typedef struct clb_adjoint clb_adjoint;

/* Device workspace for T steps with checkpoints every K steps (pressure mode
 * only; ceil(T/K) + max(K, 2) + 4 population buffers plus small arrays). */
clb_status clb_adjoint_workspace_size(const clb_params* p, int32_t T, int32_t K, size_t* bytes);

clb_status clb_adjoint_init(const clb_params* p, int32_t T, int32_t K, void* d_workspace, size_t bytes,
                            void* hip_stream, clb_adjoint** out);

/* Run the T forward steps from the start of *p, keep the checkpoints, and
 * evaluate the loss against d_dp_target[nx] (device) and m_target (!= 0).
 * *h_loss (host, may be NULL; synchronises). */
clb_status clb_adjoint_forward(clb_adjoint* a, const double* d_dp_target, double m_target, double* h_loss);

/* Backward sweep after clb_adjoint_forward.  h_grad[4] (host):
 *   [0] dL/da, [1] dL/dA1, [2] dL/dA2, [3] dL/dr,
 * where [3] treats r as an independent parameter and [1] is dL/dr * dr/dA1
 * (dr/dA1 = -sqrt(pi/6) r^2) when r is derived from A1 (p->r NaN), else 0.
 * Synchronises. */
clb_status clb_adjoint_backward(clb_adjoint* a, double* h_grad);

/* Observables of the final state: d_dp[nx] (device, may be NULL) and the
 * outlet mass flow *h_m (host, may be NULL; synchronises). */
clb_status clb_adjoint_observables(clb_adjoint* a, double* d_dp, double* h_m);

/* Post-collision populations after the T forward steps, [9][ny][nx] (device). */
clb_status clb_adjoint_final_state(clb_adjoint* a, double* d_out);

/* One reverse step for an arbitrary state: given P_n and lambda_{n+1} (both
 * [9][ny][nx], device), write lambda_n = (dP_{n+1}/dP_n)^T lambda_{n+1} and
 * h_grad3 = lambda_{n+1} . dP_{n+1}/d(a, A2, r) (host, may be NULL).
 * Does not disturb a completed forward run. */
clb_status clb_adjoint_vjp_step(clb_adjoint* a, const double* d_P, const double* d_lam_next, double* d_lam_prev,
                                double* h_grad3);

/* Release the host context (synchronises the stream first). */
clb_status clb_adjoint_destroy(clb_adjoint* a);

/* Measurement support (not part of the method): a plain device-to-device
 * copy of `bytes` bytes, one 16-byte non-temporal load and store per
 * thread, enqueued on hip_stream.  Timed, it gives the HBM bandwidth a streaming kernel reaches
 * on the GPU at hand -- the practical ceiling beside the 8 TB/s peak against
 * which the step kernels are read -- and its FETCH_SIZE / WRITE_SIZE
 * counters calibrate the traffic counters (exactly `bytes` read and written).
 * d_src, d_dst: device memory, 16-byte aligned, not overlapping; bytes a
 * multiple of 16 (0: nothing to do).  CLB_EINVAL otherwise. */
clb_status clb_hbm_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* clb_last_error(void);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif
#endif /* CLB_H */
