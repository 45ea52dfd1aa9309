/*
 * clb3d.h -- C ABI of the 3-D cascaded lattice Boltzmann step for
 * force-driven gas flow in a rectangular microduct (MI355X, gfx950).
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
 * (at a duct edge the reflection reverses both normal components); x
 * periodic (force driven, Section 3.1).
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
 * (a = 2, sigma = 1, B2 = 0.55, bulk rate 1.1, s8 = 1.2). */
typedef struct clb3_params {
  int32_t nx, ny, nz;    /* fluid nodes along the duct, across its height, across its width (>= 1) */
  int32_t zbc;           /* clb3_zbc                                                        */
  int32_t init;          /* CLB_INIT_UNIFORM (f^eq(rho0, 0)) or CLB_INIT_PERTURBED (plus
                            init_amp (2U - 1), U the top 53 bits of SplitMix64 of
                            seed XOR (27 * ((z * ny + y) * nx + x) + i), times 2^-53)     */
  int32_t cbbsr_shift;   /* Eq. 20 specular source: 1 = displaced along the walls (default);
                            0 = the node itself, z-periodic channels only (at duct edges it
                            does not conserve mass)                                         */
  double kn;             /* Knudsen number of the height H = ny, > 0          Eq. 18         */
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
} clb3_params;

typedef struct clb3_ctx clb3_ctx;

void clb3_params_default(clb3_params* p);

/* Validate *p and derive A1, r, tau_tilde, s_nu, s_q (Eqs. 18, 21 with
 * N = ny).  Host only.  CLB_EINVAL names the first invalid field. */
clb_status clb3_derive(const clb3_params* p, clb_derived* out);

/* Device workspace in bytes: two population buffers (216 bytes per node,
 * rows padded to whole segments of the device layout) plus reduction
 * scratch. */
clb_status clb3_workspace_size(const clb3_params* p, size_t* bytes);

/* Create a context over the caller's workspace (device memory, 8-byte
 * aligned, kept alive until clb3_destroy) and enqueue the start on
 * hip_stream. */
clb_status clb3_init(const clb3_params* p, void* d_workspace, size_t bytes, void* hip_stream, clb3_ctx** out);

/* Advance nsteps >= 0 steps (Eqs. 5, 20 carried to 3-D, then the collision). */
clb_status clb3_step(clb3_ctx* c, int64_t nsteps);

/* Steps taken since clb3_init / the last clb3_set_populations. */
clb_status clb3_steps_done(const clb3_ctx* c, int64_t* h_steps);

/* Density and velocity (rho u = sum e f + rho F / 2, Eqs. 12-13) of the
 * current pre-collision state, device arrays [nz][ny][nx]; any may be NULL. */
clb_status clb3_moments(clb3_ctx* c, double* d_rho, double* d_ux, double* d_uy, double* d_uz);

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
