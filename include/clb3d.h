/*
 * clb3d.h -- C ABI of the 3-D cascaded lattice Boltzmann step for
 * force-driven or pressure-driven gas flow in a rectangular microduct
 * (MI355X, gfx950).
 *
 * The paper (Liu & He, arXiv:1603.01955) develops its cascaded scheme in 2-D
 * and names the extension to rectangular ducts as future work (Section 4).
 * This step carries the 2-D method over: D3Q27 velocities; the collision of
 * Eqs. (6)-(9) read as relaxation of the central moments about the velocity
 * of Eq. (13) (trace at the bulk rate s_b, deviator and shear at s_nu of
 * Eq. 18, the seven third-order moments at s_q of Eq. 21, orders four to six
 * at s8, first order shifted by rho F as by the source of Eq. 9); the
 * combined bounce-back / specular wall of Eq. (20) on the duct walls, with
 * the reflected population taken from the node displaced along the walls
 * (at a duct edge the reflection reverses both normal components).  Two
 * kinds of duct:
 *  - force driven (xbc = CLB_X_PERIODIC, Section 3.1): x periodic, body
 *    acceleration (gx, gy, gz), the rates of Eqs. (18), (21) at Kn;
 *  - pressure driven (xbc = CLB_X_PRESSURE, Section 3.2): no force; ghost
 *    planes x = -1 and x = nx hold, for every row (y, z) of the
 *    cross-section, f^eq(2 rho_b - rho_1, 2 u_1 - u_2) + f_1 - f^eq(rho_1, u_1)
 *    (rho_1, u_1, f_1 of the column next to the plane, u_2 of the one after
 *    it, rho_b = p_ratio rho_out at the inlet, rho_out at the outlet; the
 *    2-D inlet/outlet rule row by row), and a pull or displaced specular
 *    source beyond the inlet or outlet takes the ghost value; the rates of
 *    cross-section x follow from the local Knudsen number
 *    Kn rho_out / rho_c(x), rho_c the pre-collision density at the centre of
 *    the cross-section (the mean over the middle row, or the two middle
 *    rows, of the middle layer, or the two middle layers), with N = ny in
 *    Eq. (18); the bulk rate stays s_b.
 * The D3Q27 equilibrium is the product over the axes of 2/3 - u^2 (e = 0)
 * and (1/3 + u^2 + e u) / 2 (e = +-1), times rho.
 *
 * Conventions (as in clb.h): lattice units, FP64, the caller owns device
 * memory and the stream, every call returns a clb_status and enqueues its
 * work asynchronously unless it writes a host pointer.
 *  - Grid: nx x ny x nz fluid nodes; walls half a spacing outside rows
 *    y = 0, ny - 1 (height H = ny, the N of Eq. 18) and, for a duct, layers
 *    z = 0, nz - 1 (width W = nz); z may instead be periodic (a channel).
 *  - Populations: FP64, [27][nz][ny][nx], x fastest; direction
 *    i = (a + 1) + 3 (b + 1) + 9 (c + 1) has velocity (a, b, c),
 *    a, b, c in {-1, 0, 1} (i = 13 at rest).  The stored state is the
 *    post-collision population; a step is streaming with the walls, then the
 *    collision.
 */
#ifndef CLB3D_H
#define CLB3D_H

#include "clb.h"

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

typedef enum clb3_zbc {
  CLB3_Z_WALLS = 0,     /* rectangular duct: walls below z = 0 and above z = nz - 1 */
  CLB3_Z_PERIODIC = 1   /* channel: z periodic                                      */
} clb3_zbc;

/* Problem statement; clb3_params_default fills the values of Section 3
 * (a = 2, sigma = 1, B2 = 0.55, bulk rate 1.1, s8 = 1.2; force driven;
 * p_ratio = 2, rho_out = 1 for a pressure-driven duct). */
typedef struct clb3_params {
  int32_t nx, ny, nz;    /* fluid nodes along the duct, across its height, across its width (>= 1) */
  int32_t zbc;           /* clb3_zbc                                                        */
  int32_t init;          /* CLB_INIT_UNIFORM (f^eq(rho0, 0)) or CLB_INIT_PERTURBED (plus
                            init_amp (2U - 1), U the top 53 bits of SplitMix64 of
                            seed XOR (27 * ((z * ny + y) * nx + x) + i), times 2^-53)     */
  int32_t cbbsr_shift;   /* Eq. 20 specular source: 1 = displaced along the walls (default);
                            0 = the node itself, z-periodic channels only (at duct edges it
                            does not conserve mass)                                         */
  int32_t xbc;           /* clb_xbc: CLB_X_PERIODIC (force driven, default) or CLB_X_PRESSURE
                            (pressure driven: nx >= 2, gx = gy = gz = 0; the init kind may
                            also be CLB_INIT_LINEAR_RHO, f^eq(rho(x), 0) with rho falling
                            linearly from p_ratio rho_out at x = 0 to rho_out at x = nx,
                            node centres at x + 1/2)                                        */
  double kn;             /* Knudsen number of the height H = ny (outlet Kn_out when pressure
                            driven), > 0                                      Eq. 18         */
  double a;              /* Bosanquet rarefaction factor, >= 0                Eq. 16         */
  double sigma;          /* TMAC in (0, 2]; A1 = (1 - 0.1817 sigma)(2 - sigma)/sigma if A1 NaN */
  double A1;             /* first-order slip coefficient; NaN -> from sigma                   */
  double A2;             /* second-order slip coefficient B2, >= 0            Eq. 21         */
  double r;              /* bounce-back fraction in [0, 1]; NaN -> Eq. 21 from A1              */
  double s_b, s8;        /* bulk rate and rate of orders 4-6, in (0, 2)                        */
  double gx, gy, gz;     /* body acceleration                                 Eq. 9          */
  double rho0;           /* density of the start, > 0                                           */
  double init_amp;       /* perturbation amplitude (CLB_INIT_PERTURBED), >= 0                   */
  uint64_t seed;         /* perturbation seed                                                   */
  double tq_den;         /* denominator of Eq. 21 (16 as printed)                               */
  double p_ratio;        /* p_in / p_out (pressure driven), > 0               Sec. 3.2       */
  double rho_out;        /* outlet density (pressure driven), > 0; p = rho / 3                  */
} clb3_params;

typedef struct clb3_ctx clb3_ctx;

void clb3_params_default(clb3_params* p);

/* Validate *p and derive A1, r, tau_tilde, s_nu, s_q (Eqs. 18, 21 with
 * N = ny; for a pressure-driven duct at the outlet Kn, each cross-section's
 * own rates following from its local Kn during the step).  Host only.
 * CLB_EINVAL names the first invalid field. */
clb_status clb3_derive(const clb3_params* p, clb_derived* out);

/* Device workspace in bytes: two population buffers (216 bytes per node,
 * rows padded to whole segments of the device layout), reduction scratch,
 * 67 doubles per column and, for a pressure-driven duct, the two ghost
 * planes (432 bytes per row of the cross-section). */
clb_status clb3_workspace_size(const clb3_params* p, size_t* bytes);

/* Create a context over the caller's workspace (device memory, 8-byte
 * aligned, kept alive until clb3_destroy) and enqueue the start on
 * hip_stream. */
clb_status clb3_init(const clb3_params* p, void* d_workspace, size_t bytes, void* hip_stream, clb3_ctx** out);

/* Advance nsteps >= 0 steps (Eqs. 5, 20 carried to 3-D, then the collision;
 * a pressure-driven duct first builds the ghost planes and the rates of
 * every cross-section from the state, three launches per step). */
clb_status clb3_step(clb3_ctx* c, int64_t nsteps);

/* Launch-overhead control for small ducts (a pressure-driven duct launches
 * three kernels per step): with steps_per_graph in [1, 100000], clb3_step
 * replays a hipGraph of steps_per_graph recorded steps (recorded on first
 * use from each buffer parity, on a private stream, and replayed on the
 * context's stream) and launches any remainder directly; 0 (default)
 * disables it.  Results are identical either way.  Synchronises the stream
 * when the setting changes.  CLB_EINVAL outside [0, 100000]. */
clb_status clb3_set_graph_steps(clb3_ctx* c, int32_t steps_per_graph);

/* Steps taken since clb3_init / the last clb3_set_populations. */
clb_status clb3_steps_done(const clb3_ctx* c, int64_t* h_steps);

/* Density and velocity (rho u = sum e f + rho F / 2, Eqs. 12-13) of the
 * current pre-collision state, device arrays [nz][ny][nx]; any may be NULL. */
clb_status clb3_moments(clb3_ctx* c, double* d_rho, double* d_ux, double* d_uy, double* d_uz);

/* Mass flow through each cross-section (Section 3.2 carried to the duct):
 * m(x) = sum_{y,z} rho u_x of the current pre-collision state
 * (rho u_x = sum e_x f + rho gx / 2).  Optional per-column d_m_col[nx]
 * (device); *h_m_mean (host, may be NULL) receives the mean over x and then
 * the call synchronises.  Fixed summation order. */
clb_status clb3_massflow(clb3_ctx* c, double* d_m_col, double* h_m_mean);

/* Pressure deviation along the duct's centre line (Section 3.2):
 * d_dp[x] = (p_c(x) - p_l(x)) / p_out, p_c = rho_c / 3 at the centre of the
 * cross-section (as for the local Knudsen number), p_l falling linearly from
 * p_in at x = 0 to p_out at x = nx (node centres x + 1/2); optional
 * d_rho_c[x].  Device arrays of nx doubles, either may be NULL.
 * Pressure-driven ducts only (CLB_ESTATE otherwise). */
clb_status clb3_pressure_deviation(clb3_ctx* c, double* d_dp, double* d_rho_c);

/* Dimensionless flow rate of Section 3.1 carried to the duct:
 * Q = sqrt(6) sum_{y,z} u_x / (3 gx H^2 W), averaged over x (for a z-periodic
 * channel the 2-D Q).  Needs gx != 0.  Synchronises. */
clb_status clb3_flow_rate(clb3_ctx* c, double* h_Q);

/* Copy the post-collision populations out / in ([27][nz][ny][nx], device;
 * converted from / to the library's own device layout).  Setting them
 * resets the step counter. */
clb_status clb3_get_populations(clb3_ctx* c, double* d_out);
clb_status clb3_set_populations(clb3_ctx* c, const double* d_in);

/* *h_ok = 1 if every population is finite, else 0 and CLB_EUNSTABLE.
 * Synchronises. */
clb_status clb3_check_finite(clb3_ctx* c, int32_t* h_ok);

/* Release the host context (not the workspace or the stream). */
clb_status clb3_destroy(clb3_ctx* c);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif
#endif /* CLB3D_H */
