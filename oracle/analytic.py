"""Closed-form steady solutions that pin the CLB reference (test infrastructure).

All formulas follow from the paper's equations; the derivations are sketched
next to each function so that a reader can redo them.

Notation: H = N = ny fluid rows between half-way walls; g the body
acceleration; tt = s_nu^-1 - 1/2 (Eq. 18), so the kinematic viscosity is
nu = tt/3 (Eq. 14 with c_s^2 = 1/3); tau_q = 1/s_q (Eq. 21); r the CBBSR
bounce-back fraction (Eq. 20); A1 = B1 sigma_v and B2 the slip coefficients
of Eq. (19); lambda_e = sqrt(pi/6) tt the effective mean free path
(Eqs. 15-17 with RT = 1/3, mu_e = rho nu).
"""
from math import pi, sqrt

from .clb_ref import tau_tilde, rate_q


# ---------------------------------------------------------------------------
# Discrete steady force-driven channel (periodic, x-uniform, F = (g, 0)).
#
# Derivation sketch.  For an x-uniform steady state, linear in g, only the
# x-odd/y-even combinations A = f1 - f3, B = f5 - f6, C = f8 - f7 carry the
# flow; they give the raw moments k_x = A + B + C, k_xy = B - C and
# k_xyy = B + C.  Linearising Eq. (7) about rest: the x-momentum gains g per
# step (Eqs. 4, 9), k_xy relaxes at s_nu, and k_xyy relaxes towards u/3 at
# s_q (the forcing of Eq. (9) has no second- or higher-order central
# moments).  Pull streaming moves B up and C down one row; the bottom wall of
# Eq. (20) gives B_0 = (1 - 2r) C~_0 (mirror image at the top).  Solving the
# resulting three-term recurrences gives a velocity that is exactly a
# parabola in the bulk, u(y) = U_s + G y (H - y) with G = g / (2 nu) and
# y = j + 1/2, and the wall equation fixes the slip
#   U_s = (3/2) ((1 - r)/r) g H + 3 g (4 tau_s - 3)/(8 tt) + 3 g (tau_q - 1),
# tau_s = tt + 1/2.  (With r = 1 and (tau_s - 1/2)(tau_q - 1/2) = 1/8 the
# slip vanishes: the classic "magic" combination for this forcing.)
# ---------------------------------------------------------------------------
def discrete_channel(N, kn, a, A2, r, g, tq_den=16.0):
    """Returns (U_s, G, u_rows, sum_u) of the steady discrete solution."""
    tt = tau_tilde(kn, N, a)
    tau_s = tt + 0.5
    tau_q = 1.0 / rate_q(kn, N, a, A2, tq_den)
    G = 3.0 * g / (2.0 * tt)
    U_s = (1.5 * (1.0 - r) / r * g * N + 3.0 * g * (4.0 * tau_s - 3.0) / (8.0 * tt)
           + 3.0 * g * (tau_q - 1.0))
    rows = [U_s + G * (j + 0.5) * (N - (j + 0.5)) for j in range(N)]
    sum_u = N * U_s + G * (N ** 3 / 6.0 + N / 12.0)
    return U_s, G, rows, sum_u


def discrete_Q(N, kn, a, A2, r, tq_den=16.0):
    """Dimensionless flow rate of Section 3.1 for the discrete steady channel:
    Q = sqrt(6) sum_y u / (3 g H^2)  (independent of g in the linear regime)."""
    _, _, _, sum_u = discrete_channel(N, kn, a, A2, r, 1.0, tq_den)
    return sqrt(6.0) * sum_u / (3.0 * N * N)


# ---------------------------------------------------------------------------
# Continuum Poiseuille flow with the modified second-order slip law Eq. (19):
# u = U_s + G y (H - y) with du/dn|_w = G H and d2u/dn2 = -2 G, so
#   U_s = A1 lambda_e G H + 2 B2 lambda_e^2 G
#       = (3/2) A1 sqrt(pi/6) g H + (pi/2) B2 tt g.
# The discrete scheme reproduces the first-order part exactly through r of
# Eq. (21); its second-order part equals this one when the Eq. (21)
# denominator is 24, and exceeds it by 3 g/(16 tt) + (pi/4) B2 tt g with the
# printed 16.
# ---------------------------------------------------------------------------
def continuum_slip(N, kn, a, A1, A2, g):
    tt = tau_tilde(kn, N, a)
    return 1.5 * A1 * sqrt(pi / 6.0) * g * N + 0.5 * pi * A2 * tt * g


def continuum_sum_u(N, kn, a, A1, A2, g):
    tt = tau_tilde(kn, N, a)
    G = 3.0 * g / (2.0 * tt)
    return N * continuum_slip(N, kn, a, A1, A2, g) + G * (N ** 3 / 6.0 + N / 12.0)


# ---------------------------------------------------------------------------
# Knudsen minimum.  For large N with k_e = Kn/(1 + a Kn), tt = sqrt(6/pi) N k_e
# and the discrete Q above tends to
#   Q(Kn) = (sqrt(pi)/2) [A1 + 1/(6 k_e) + 3 B2 k_e]      (printed 16 in Eq. 21)
# which is smallest at k_e = 1/sqrt(18 B2), i.e. Kn* = 1/(sqrt(18 B2) - a).
# (The continuum law would have 2 B2 in place of 3 B2.)
# ---------------------------------------------------------------------------
def large_N_Q(kn, a, A1, A2):
    ke = kn / (1.0 + a * kn)
    return 0.5 * sqrt(pi) * (A1 + 1.0 / (6.0 * ke) + 3.0 * A2 * ke)


def knudsen_minimum(a, A2):
    return 1.0 / (sqrt(18.0 * A2) - a)


# ---------------------------------------------------------------------------
# Long pressure-driven channel, lubrication limit (Section 3.2).  Locally the
# flow is a fully developed channel flow with rho g = -dp/dx, p = rho/3 and a
# local Knudsen number Kn = Kn_out p_out / p, so rho Kn is constant and
# mu_e = mu/(1 + a Kn) with mu = (1/3) sqrt(6/pi) rho_out Kn_out H (Eqs. 15-18).
# The mass flow m = rho sum_y u is then
#   m = rho g H^3 / (12 nu_e) [1 + 6 A1 k_e + c2 B2 k_e^2 + 3/(4 H^2)]
# (the last term is the small discrete part of the slip), and m is the same at
# every x; integrating -dp/dx from the outlet with RK4 and choosing m so that
# p(0) = p_in gives the reference pressure profile.  The second-order slip
# coefficient c2 is 12 for the slip law of Eq. (19) itself (a parabola with
# slip u_s = A1 lambda_e u' - A2 lambda_e^2 u'' carries
# 1 + 6 A1 k_e + 12 A2 k_e^2 times the no-slip flow) and 18 for the
# force-driven periodic channel above, whose body-force source adds the
# discrete excess of half of B2 (discrete_channel).  A pressure-driven channel
# has no body force; its steady states follow c2 = 12.
# ---------------------------------------------------------------------------
def lubrication_profile(nx, ny, kn_out, p_ratio, a, A1, A2, rho_out=1.0, nsub=20, discrete=True, c2=18.0):
    """Returns (m, p(x_i)) at node centres x_i = i + 1/2 for the lubrication
    model; discrete=False drops the 3/(4 H^2) term (the continuum model), c2
    is the coefficient of B2 k_e^2 in the slip bracket."""
    H = float(ny)
    p_out = rho_out / 3.0
    p_in = p_ratio * p_out
    mu = sqrt(6.0 / pi) * rho_out * kn_out * H / 3.0

    def dpdx(p, m):
        kn = kn_out * p_out / p
        ke = kn / (1.0 + a * kn)
        mu_e = mu / (1.0 + a * kn)
        bracket = 1.0 + 6.0 * A1 * ke + c2 * A2 * ke * ke + (0.75 / (H * H) if discrete else 0.0)
        # m = rho (-dp/dx) H^3 / (12 mu_e) * bracket / rho ... with rho = 3 p:
        # m = 3 p (-dp/dx) H^3 bracket / (12 mu_e)
        return -12.0 * mu_e * m / (3.0 * p * H ** 3 * bracket)

    def integrate(m, xs):
        # march from the outlet (x = L) towards the inlet (x = 0) with RK4
        L = float(nx)
        out = {}
        p = p_out
        x = L
        targets = sorted(xs, reverse=True)
        h = L / (nx * nsub)
        ti = 0
        while ti < len(targets) and targets[ti] >= x - 1e-12:
            out[targets[ti]] = p
            ti += 1
        while x > 1e-12:
            step = min(h, x)
            k1 = dpdx(p, m)
            k2 = dpdx(p - 0.5 * step * k1, m)
            k3 = dpdx(p - 0.5 * step * k2, m)
            k4 = dpdx(p - step * k3, m)
            p = p - step * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
            x -= step
            while ti < len(targets) and targets[ti] >= x - 1e-9:
                out[targets[ti]] = p
                ti += 1
        return p, out

    lo, hi = 0.0, 1.0
    while integrate(hi, [])[0] < p_in:
        hi *= 2.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if integrate(mid, [])[0] < p_in:
            lo = mid
        else:
            hi = mid
    m = 0.5 * (lo + hi)
    xs = [i + 0.5 for i in range(nx)]
    _, prof = integrate(m, xs)
    return m, [prof[x] for x in xs]


# ---------------------------------------------------------------------------
# Continuum no-slip mass flow of the long channel, the m_ns of the
# dimensionless mass flow S = m / m_ns in Section 3.2.  Without rarefaction
# the gas has its plain viscosity mu (Eq. 17 without the Bosanquet factor,
# mu = (1/3) sqrt(6/pi) rho Kn H, the same at every x because rho Kn is
# constant) and sticks to the walls, so locally m = rho H^3 (-dp/dx) / (12 mu)
# (plane Poiseuille flow) with rho = p / RT, RT = 1/3.  m is the same at
# every x, so m dx = -(H^3 / (12 mu RT)) p dp integrates from inlet to outlet
# to  m_ns = H^3 (p_in^2 - p_out^2) / (24 mu RT L).
# ---------------------------------------------------------------------------
def noslip_massflow(nx, ny, kn_out, p_ratio, rho_out=1.0):
    H, L = float(ny), float(nx)
    RT = 1.0 / 3.0
    p_out = rho_out * RT
    p_in = p_ratio * p_out
    mu = sqrt(6.0 / pi) * rho_out * kn_out * H / 3.0
    return H ** 3 * (p_in * p_in - p_out * p_out) / (24.0 * mu * RT * L)
