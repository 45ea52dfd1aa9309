"""Plain NumPy FP64 reference of the CLB time step (test infrastructure only).

Not part of the product path: only tests, the smoke check and the CPU-baseline
leg of the benchmark may import it.  It is written for a reader to check
against the paper by eye, not for speed.  Every function is dtype-generic
(real or complex: no abs(), no comparisons on state values), so the same code
can be run in complex128 for complex-step derivatives.

State convention: ``P`` holds the post-collision transformed populations
(the tilde-bar f of Eq. 4), shape (9, ny, nx), x fastest.  One step is
``pre = stream_bc(P)`` (Eqs. 5 and 20 plus the x boundaries) followed by
``P = collide(pre)`` (Eq. 4).  Fluid row y sits at height y + 1/2; the walls
lie half a spacing outside rows 0 and ny-1, so H = ny lattice units.

Readings of points the paper leaves open (each is also listed in the design
notes):
  * F is an acceleration g; the body-force density is rho*g (Eqs. 9, 13).
  * The lattice number N of Eq. (18) is the number of fluid rows ny.
  * Eq. (20) specular part: geometric neighbour x-1 / x+1 (cbbsr_shift=1) or
    the same node (cbbsr_shift=0).  Top wall = mirror image of the bottom.
  * Pressure inlet/outlet (Section 3.2 cites an external scheme whose details
    are not in the paper): ghost columns at x=-1 and x=nx, built each step
    from the post-collision populations of the two adjacent columns:
    rho_g = 2 rho_b - rho_1, u_g = 2 u_1 - u_2,
    f_g = f^eq(rho_g, u_g) + (f_1 - f^eq(rho_1, u_1)).   Parity unpinned
    against the paper (no numbers in the paper fix it).
  * Local Kn (Section 3.2): Kn(x) = Kn_out rho_out / rho_c(x), rho_c the
    centre-line density of the same step's pre-collision state (mean of the
    two middle rows for even ny).
  * Eq. (21) denominator 16 by default; 24 available as a variant.
"""
import dataclasses
from math import pi, sqrt
from typing import Optional

import numpy as np

from .lattice import EX, EY, T, T_INV, central_shift, feq
from .rng import uniform01

SQRT_6_OVER_PI = sqrt(6.0 / pi)
SQRT_PI_OVER_6 = sqrt(pi / 6.0)


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    xbc: str = "periodic"          # "periodic" (Section 3.1) or "pressure" (Section 3.2)
    kn: complex = 0.1              # Kn (periodic) or Kn_out (pressure)
    a: complex = 2.0               # Bosanquet rarefaction factor, Eq. (16), Section 3
    sigma: float = 1.0             # TMAC, Eq. (19)
    A1: Optional[complex] = None   # B1*sigma_v; None -> from sigma (Eq. 19, Section 3)
    A2: complex = 0.55             # B2, Section 3
    r: Optional[complex] = None    # bounce-back fraction; None -> Eq. (21)
    s3: float = 1.1                # Section 3
    s8: float = 1.2                # Section 3
    gx: float = 0.0                # body acceleration (periodic mode)
    gy: float = 0.0
    p_ratio: float = 2.0           # p_in / p_out (pressure mode)
    rho_out: float = 1.0
    rho0: float = 1.0
    ux0: float = 0.0
    uy0: float = 0.0
    tq_den: float = 16.0           # Eq. (21) denominator (16 as printed)
    cbbsr_shift: int = 1
    forcing: int = 0               # 0: source of Eq. (9); 1: plus third-order moments (see collide)


# ---------------------------------------------------------------------------
# Parameters: Eqs. (14)-(18), (19), (21) and the values listed in Section 3.
# ---------------------------------------------------------------------------
def slip_A1(sigma):
    """A1 = B1 * sigma_v with B1 = 1 - 0.1817 sigma (Section 3) and
    sigma_v = (2 - sigma)/sigma (after Eq. 19)."""
    return (1.0 - 0.1817 * sigma) * (2.0 - sigma) / sigma


def bounce_fraction(A1):
    """Eq. (21): r_b = 1 / (1 + B1 sigma_v sqrt(pi/6))."""
    return 1.0 / (1.0 + A1 * SQRT_PI_OVER_6)


def tau_tilde(kn, N, a):
    """Eq. (18) minus one half: s_nu^-1 - 1/2 = sqrt(6/pi) N Kn / (1 + a Kn)."""
    return SQRT_6_OVER_PI * N * kn / (1.0 + a * kn)


def rate_nu(kn, N, a):
    """Eq. (18): shear relaxation rate s_nu."""
    return 1.0 / (0.5 + tau_tilde(kn, N, a))


def rate_q(kn, N, a, A2, den=16.0):
    """Eq. (21): s_q^-1 = 1/2 + (3 + 4 pi tt^2 B2) / (den tt), tt = s_nu^-1 - 1/2."""
    tt = tau_tilde(kn, N, a)
    return 1.0 / (0.5 + (3.0 + 4.0 * pi * tt * tt * A2) / (den * tt))


def resolved(prm):
    """(A1, r) actually used: explicit values win over the sigma-derived ones."""
    A1 = prm.A1 if prm.A1 is not None else slip_A1(prm.sigma)
    r = prm.r if prm.r is not None else bounce_fraction(A1)
    return A1, r


def rho_in(prm):
    return prm.p_ratio * prm.rho_out


# ---------------------------------------------------------------------------
# Initial states (the paper gives none; uniform rest state, linear density
# for the long channel, and a seeded perturbation of the equilibrium).
# ---------------------------------------------------------------------------
def init_uniform(prm, dtype=np.float64):
    f = feq(np.full((prm.ny, prm.nx), prm.rho0, dtype=dtype), prm.ux0, prm.uy0)
    return np.ascontiguousarray(f)


def x_positions(prm):
    """Node centres x_i = i + 1/2; inlet plane at x = 0, outlet at x = L = nx."""
    return np.arange(prm.nx, dtype=np.float64) + 0.5


def init_linear_rho(prm, dtype=np.float64):
    L = float(prm.nx)
    rin = rho_in(prm)
    rho_x = rin - (rin - prm.rho_out) * x_positions(prm) / L
    rho = np.broadcast_to(rho_x, (prm.ny, prm.nx)).astype(dtype)
    return np.ascontiguousarray(feq(rho, 0.0, 0.0))


def init_perturbed(prm, seed, amp):
    """P_i = f_i^eq(rho0, u0) + amp (2U - 1), U from SplitMix64 keyed by
    seed XOR (9 * node + i), node = y * nx + x."""
    P = init_uniform(prm)
    node = np.arange(prm.ny * prm.nx, dtype=np.uint64).reshape(prm.ny, prm.nx)
    for i in range(9):
        U = uniform01(seed, np.uint64(9) * node + np.uint64(i))
        P[i] += amp * (2.0 * U - 1.0)
    return P


def init_perturbed_rows(prm, seed, amp, y0, y1):
    """Rows y0 .. y1 - 1 (full width) of init_perturbed: the same generator
    keyed by the same node numbers, evaluated for those rows only (grids too
    large to hold whole)."""
    P = init_uniform(dataclasses.replace(prm, ny=y1 - y0))
    node = (np.arange(y0, y1, dtype=np.uint64)[:, None] * np.uint64(prm.nx)
            + np.arange(prm.nx, dtype=np.uint64)[None, :])
    for i in range(9):
        U = uniform01(seed, np.uint64(9) * node + np.uint64(i))
        P[i] += amp * (2.0 * U - 1.0)
    return P


# ---------------------------------------------------------------------------
# Macroscopic quantities, Eqs. (12)-(13): rho = sum f, rho u = sum e f + rho F/2.
# ---------------------------------------------------------------------------
def macroscopic(f, gx=0.0, gy=0.0):
    rho = f.sum(axis=0)
    jx = np.tensordot(EX.astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(EY.astype(np.float64), f, axes=(0, 0))
    return rho, jx / rho + 0.5 * gx, jy / rho + 0.5 * gy


# ---------------------------------------------------------------------------
# x boundaries: periodic wrap (Section 3.1) or pressure ghost columns
# (Section 3.2; see the module docstring for the reading adopted).
# ---------------------------------------------------------------------------
def _pressure_ghost(f_adj, f_adj2, rho_b):
    rho1, ux1, uy1 = macroscopic(f_adj)
    _, ux2, uy2 = macroscopic(f_adj2)
    rho_g = 2.0 * rho_b - rho1
    ux_g = 2.0 * ux1 - ux2
    uy_g = 2.0 * uy1 - uy2
    return feq(rho_g, ux_g, uy_g) + (f_adj - feq(rho1, ux1, uy1))


def ghost_columns(P, prm):
    """Populations of the columns x = -1 and x = nx, each of shape (9, ny)."""
    if prm.xbc == "periodic":
        return P[:, :, -1], P[:, :, 0]
    if prm.xbc == "pressure":
        g_in = _pressure_ghost(P[:, :, 0], P[:, :, 1], rho_in(prm))
        g_out = _pressure_ghost(P[:, :, -1], P[:, :, -2], prm.rho_out)
        return g_in, g_out
    raise ValueError(prm.xbc)


# ---------------------------------------------------------------------------
# Streaming (Eq. 5) with the CBBSR walls (Eq. 20) -> pre-collision f-bar.
# ---------------------------------------------------------------------------
def stream_bc(P, prm, r=None):
    if r is None:
        r = resolved(prm)[1]
    _, ny, nx = P.shape
    g_in, g_out = ghost_columns(P, prm)
    # Extended array: column c + 1 holds x = c; column 0 is x = -1, column nx + 1 is x = nx.
    Pext = np.concatenate([g_in[:, :, None], P, g_out[:, :, None]], axis=2)
    pre = np.empty_like(P)
    for i in range(9):
        ex, ey = int(EX[i]), int(EY[i])
        cols = slice(1 - ex, 1 - ex + nx)          # source column x - e_x
        if ey == 0:
            pre[i] = Pext[i, :, cols]
        elif ey == 1:                              # source row y - 1
            pre[i, 1:] = Pext[i, :-1, cols]
        else:                                      # source row y + 1
            pre[i, :-1] = Pext[i, 1:, cols]
    # Bottom wall (half a spacing below row 0): unknowns 2, 5, 6.
    b = 0
    spec5 = Pext[8, b, 0:nx] if prm.cbbsr_shift else P[8, b]      # f8 from x-1
    spec6 = Pext[7, b, 2:nx + 2] if prm.cbbsr_shift else P[7, b]  # f7 from x+1
    pre[2, b] = P[4, b]
    pre[5, b] = r * P[7, b] + (1.0 - r) * spec5
    pre[6, b] = r * P[8, b] + (1.0 - r) * spec6
    # Top wall (mirror y -> -y: 2<->4, 5<->8, 6<->7): unknowns 4, 7, 8.
    t = ny - 1
    spec7 = Pext[6, t, 2:nx + 2] if prm.cbbsr_shift else P[6, t]  # f6 from x+1
    spec8 = Pext[5, t, 0:nx] if prm.cbbsr_shift else P[5, t]      # f5 from x-1
    pre[4, t] = P[2, t]
    pre[7, t] = r * P[5, t] + (1.0 - r) * spec7
    pre[8, t] = r * P[6, t] + (1.0 - r) * spec8
    return pre


def gather_nodes(P, prm, ys, xs, r=None):
    """Pre-collision populations at selected nodes only (periodic x), by
    direct neighbour lookup; shape (9, len(ys)).  Used to check single nodes
    of grids too large to step whole."""
    if prm.xbc != "periodic":
        raise ValueError("gather_nodes supports periodic x only")
    if r is None:
        r = resolved(prm)[1]
    _, ny, nx = P.shape
    ys = np.asarray(ys)
    xs = np.asarray(xs)
    out = np.empty((9, ys.size), dtype=P.dtype)
    for i in range(9):
        sy = np.clip(ys - EY[i], 0, ny - 1)        # clipped rows are overwritten below
        sx = (xs - EX[i]) % nx
        out[i] = P[i, sy, sx]
    xm = (xs - 1) % nx
    xp = (xs + 1) % nx
    bot = ys == 0
    top = ys == ny - 1
    sh = bool(prm.cbbsr_shift)
    out[2, bot] = P[4, 0, xs[bot]]
    out[5, bot] = r * P[7, 0, xs[bot]] + (1 - r) * P[8, 0, (xm if sh else xs)[bot]]
    out[6, bot] = r * P[8, 0, xs[bot]] + (1 - r) * P[7, 0, (xp if sh else xs)[bot]]
    out[4, top] = P[2, ny - 1, xs[top]]
    out[7, top] = r * P[5, ny - 1, xs[top]] + (1 - r) * P[6, ny - 1, (xp if sh else xs)[top]]
    out[8, top] = r * P[6, ny - 1, xs[top]] + (1 - r) * P[5, ny - 1, (xm if sh else xs)[top]]
    return out


# ---------------------------------------------------------------------------
# Collision, form 1 (the one the time stepper uses): explicit moment matrices.
# Raw moments M = T f (Eq. 10); central moments about the physical velocity
# kappa = N(u) M; orders 2-4 relax towards the central moments of the
# equilibrium (Eq. 11: kxx+kyy = 2 rho/3, kxxyy = rho/9, the rest 0) at the
# rates s3, s4=s5=s_nu, s6=s7=s_q, s8 (Eq. 14, Section 3); the force shifts
# the first-order central moments by rho F (Eqs. 4, 9, 13); back-transform
# f = T^-1 N(-u) kappa'.
# ---------------------------------------------------------------------------
def _apply(mats, vecs):
    """Per-node matrix-vector products: mats (n, 9, 9), vecs (9, n) -> (9, n)."""
    return np.matmul(mats, vecs.T[:, :, None])[:, :, 0].T


def collide(pre, gx, gy, s3, s_nu, s_q, s8, forcing=0):
    """forcing=1 adds (1 - s_q/2) rho F/3 to the post-collision raw moments
    k_xxy (F_y) and k_xyy (F_x): the third-order moments of the second-order
    (Guo-type) discrete force term with its usual (1 - s/2) factor, which the
    source of Eq. (9) leaves out.  With them the printed Eq. (21) is the exact
    match to the slip law of Eq. (19) in a force-driven channel."""
    shape = pre.shape
    f = pre.reshape(9, -1)
    M = T @ f
    rho = M[0]
    ux = M[1] / rho + 0.5 * gx
    uy = M[2] / rho + 0.5 * gy
    kap = _apply(central_shift(ux, uy), M)
    n = f.shape[1]
    rates = {
        3: np.broadcast_to(s3, shape[1:]).reshape(n),
        4: np.broadcast_to(s_nu, shape[1:]).reshape(n),
        5: np.broadcast_to(s_nu, shape[1:]).reshape(n),
        6: np.broadcast_to(s_q, shape[1:]).reshape(n),
        7: np.broadcast_to(s_q, shape[1:]).reshape(n),
        8: np.broadcast_to(s8, shape[1:]).reshape(n),
    }
    kap_eq = np.zeros_like(kap)
    kap_eq[3] = 2.0 / 3.0 * rho
    kap_eq[8] = rho / 9.0
    post = np.empty_like(kap)
    post[0] = kap[0]
    post[1] = kap[1] + rho * gx
    post[2] = kap[2] + rho * gy
    for k in range(3, 9):
        post[k] = kap[k] - rates[k] * (kap[k] - kap_eq[k])
    M_post = _apply(central_shift(-ux, -uy), post)
    if forcing:
        third = (1.0 - 0.5 * rates[6]) * rho / 3.0
        M_post[6] = M_post[6] + third * gy
        M_post[7] = M_post[7] + third * gx
    return (T_INV @ M_post).reshape(shape)


# ---------------------------------------------------------------------------
# Collision, form 2: the closed form exactly as printed, Eqs. (6)-(9), with
# S = T^-1 S_hat.  Used to pin form 1 (they must agree to rounding).
# ---------------------------------------------------------------------------
def collide_literal(pre, gx, gy, s3, s4, s5, s6, s7, s8):
    f0, f1, f2, f3, f4, f5, f6, f7, f8 = pre
    Fx, Fy = gx, gy
    # Eq. (8): raw moments of the pre-collision f-bar.
    rho = f0 + f1 + f2 + f3 + f4 + f5 + f6 + f7 + f8
    k_x = f1 - f3 + f5 - f6 - f7 + f8
    k_y = f2 - f4 + f5 + f6 - f7 - f8
    k_xx = f1 + f3 + f5 + f6 + f7 + f8
    k_yy = f2 + f4 + f5 + f6 + f7 + f8
    k_xy = (f5 + f7) - (f6 + f8)
    k_xxy = (f5 + f6) - (f7 + f8)
    k_xyy = (f5 + f8) - (f6 + f7)
    k_xxyy = f5 + f6 + f7 + f8
    # Eq. (13)
    ux = k_x / rho + 0.5 * Fx
    uy = k_y / rho + 0.5 * Fy
    # Eq. (7)
    g3 = s3 / 12.0 * (2.0 / 3.0 * rho + rho * (ux * ux + uy * uy) - (k_xx + k_yy)
                      - 0.5 * rho * (2.0 * Fx * ux + 2.0 * Fy * uy))
    g4 = s4 / 4.0 * (rho * (ux * ux - uy * uy) - (k_xx - k_yy)
                     - 0.5 * rho * (2.0 * Fx * ux - 2.0 * Fy * uy))
    g5 = s5 / 4.0 * (rho * ux * uy - k_xy - 0.5 * rho * (Fx * uy + Fy * ux))
    g6 = (s6 / 4.0 * (2.0 * rho * ux * ux * uy + k_xxy - 2.0 * ux * k_xy - uy * k_xx
                      - 0.5 * rho * (Fy * ux * ux + 2.0 * Fx * ux * uy))
          - 0.5 * uy * (3.0 * g3 + g4) - 2.0 * ux * g5)
    g7 = (s7 / 4.0 * (2.0 * rho * ux * uy * uy + k_xyy - 2.0 * uy * k_xy - ux * k_yy
                      - 0.5 * rho * (Fx * uy * uy + 2.0 * Fy * uy * ux))
          - 0.5 * ux * (3.0 * g3 - g4) - 2.0 * uy * g5)
    g8 = (s8 / 4.0 * (rho / 9.0 + 3.0 * rho * ux * ux * uy * uy
                      - (k_xxyy - 2.0 * ux * k_xyy - 2.0 * uy * k_xxy + ux * ux * k_yy
                         + uy * uy * k_xx + 4.0 * ux * uy * k_xy)
                      - 0.5 * rho * (2.0 * Fx * ux * uy * uy + 2.0 * Fy * uy * ux * ux))
          - 2.0 * g3 - 0.5 * uy * uy * (3.0 * g3 + g4) - 0.5 * ux * ux * (3.0 * g3 - g4)
          - 4.0 * ux * uy * g5 - 2.0 * uy * g6 - 2.0 * ux * g7)
    # Eq. (9), then S = T^-1 S_hat.
    zero = 0.0 * rho
    S_hat = np.stack([
        zero,
        rho * Fx,
        rho * Fy,
        2.0 * rho * (ux * Fx + uy * Fy),
        2.0 * rho * (ux * Fx - uy * Fy),
        rho * (ux * Fy + uy * Fx),
        rho * Fy * ux * ux + 2.0 * rho * Fx * ux * uy,
        rho * Fx * uy * uy + 2.0 * rho * Fy * uy * ux,
        2.0 * rho * Fx * ux * uy * uy + 2.0 * rho * Fy * uy * ux * ux,
    ])
    S = np.tensordot(T_INV, S_hat, axes=(1, 0))
    # Eq. (6) with g0 = g1 = g2 = 0 and delta_t = 1.
    return np.stack([
        f0 - 4.0 * (g3 - g8) + S[0],
        f1 - g3 + g4 + 2.0 * (g7 - g8) + S[1],
        f2 - g3 - g4 + 2.0 * (g6 - g8) + S[2],
        f3 - g3 + g4 - 2.0 * (g7 + g8) + S[3],
        f4 - g3 - g4 - 2.0 * (g6 + g8) + S[4],
        f5 + 2.0 * g3 + g5 - g6 - g7 + g8 + S[5],
        f6 + 2.0 * g3 - g5 - g6 + g7 + g8 + S[6],
        f7 + 2.0 * g3 + g5 + g6 + g7 + g8 + S[7],
        f8 + 2.0 * g3 - g5 + g6 - g7 + g8 + S[8],
    ])


# ---------------------------------------------------------------------------
# Relaxation rates for a step.
# ---------------------------------------------------------------------------
def centre_density(rho):
    """rho_c(x) from a (ny, nx) density field: middle row (odd ny) or mean of
    the two middle rows (even ny)."""
    ny = rho.shape[0]
    if ny % 2:
        return rho[ny // 2]
    return 0.5 * (rho[ny // 2 - 1] + rho[ny // 2])


def step_rates(pre, prm):
    """(s_nu, s_q) for this step: constants (periodic), or per column from the
    local Knudsen number Kn(x) = Kn_out p_out / p_c(x) (pressure)."""
    if prm.xbc == "periodic":
        kn = prm.kn
    else:
        rho, _, _ = macroscopic(pre)
        kn = prm.kn * prm.rho_out / centre_density(rho)
    return (rate_nu(kn, prm.ny, prm.a),
            rate_q(kn, prm.ny, prm.a, prm.A2, prm.tq_den))


def step(P, prm):
    """One CLB step: P (post-collision at t-1) -> P (post-collision at t)."""
    _, r = resolved(prm)
    pre = stream_bc(P, prm, r)
    s_nu, s_q = step_rates(pre, prm)
    return collide(pre, prm.gx, prm.gy, prm.s3, s_nu, s_q, prm.s8, prm.forcing)


def run(P, prm, nsteps, callback=None):
    for n in range(nsteps):
        P = step(P, prm)
        if callback is not None:
            callback(n + 1, P)
    return P


def run_rows(P, prm, nsteps):
    """nsteps periodic steps of a band of full-width rows P (9, rows, nx) cut
    out of the channel prm: the rates of Eqs. (18), (21) use the channel's
    N = prm.ny, and both edges of the band are stepped as walls (Eq. 20).
    Where the band ends at a channel wall that is the channel's own rule; at
    a cut edge it is not, and after nsteps the rows within nsteps of a cut
    edge no longer hold the channel's values (the others do)."""
    if prm.xbc != "periodic":
        raise ValueError("run_rows supports periodic x only")
    _, r = resolved(prm)
    band = dataclasses.replace(prm, ny=P.shape[1])
    s_nu, s_q = rate_nu(prm.kn, prm.ny, prm.a), rate_q(prm.kn, prm.ny, prm.a, prm.A2, prm.tq_den)
    for _ in range(nsteps):
        P = collide(stream_bc(P, band, r), prm.gx, prm.gy, prm.s3, s_nu, s_q, prm.s8, prm.forcing)
    return P


def step_nodes(P, prm, ys, xs):
    """Post-collision populations at the selected nodes after one step from P
    (periodic x only), shape (9, len(ys))."""
    _, r = resolved(prm)
    pre = gather_nodes(P, prm, ys, xs, r)
    s_nu, s_q = step_rates(pre, prm)
    return collide(pre, prm.gx, prm.gy, prm.s3, s_nu, s_q, prm.s8, prm.forcing)


# ---------------------------------------------------------------------------
# Diagnostics (Eqs. 12-13; Sections 3.1 and 3.2).  All of them are moments of
# the pre-collision state StreamBC(P) at the current time level.
# ---------------------------------------------------------------------------
def moments(P, prm):
    pre = stream_bc(P, prm)
    g = (prm.gx, prm.gy) if prm.xbc == "periodic" else (0.0, 0.0)
    return macroscopic(pre, *g)


def column_sums(P, prm):
    """Per column x: m(x) = sum_y rho u_x (mass flow, Section 3.2),
    su(x) = sum_y u_x, and the centre-line density rho_c(x)."""
    rho, ux, _ = moments(P, prm)
    return (rho * ux).sum(axis=0), ux.sum(axis=0), centre_density(rho)


def flow_rate_Q(P, prm):
    """Dimensionless flow rate of Section 3.1:
    Q = (int u_x dy) / (F_x H^2 sqrt(RT/2) / p), with F_x = rho0 g,
    RT = 1/3 and p = rho0/3, the integral a midpoint sum over the fluid rows
    (averaged over x)."""
    _, su, _ = column_sums(P, prm)
    H = float(prm.ny)
    return su.mean() * sqrt(6.0) / (3.0 * prm.gx * H * H)


def pressure_deviation(P, prm):
    """delta p(x) = (p_c(x) - p_l(x)) / p_out with p = rho/3 and the linear
    profile p_l falling from p_in at x = 0 to p_out at x = L (Section 3.2)."""
    _, _, rho_c = column_sums(P, prm)
    p_out = prm.rho_out / 3.0
    p_in = prm.p_ratio * p_out
    L = float(prm.nx)
    p_l = p_in - (p_in - p_out) * x_positions(prm) / L
    return (rho_c / 3.0 - p_l) / p_out
