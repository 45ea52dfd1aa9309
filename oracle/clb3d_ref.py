"""Plain NumPy FP64 reference of a 3-D cascaded LB step for force-driven gas
flow in a rectangular microduct (test infrastructure only).

Not part of the product path: only tests, the smoke check and the CPU-baseline
leg of the benchmark may import it.  Written to be checked by eye, not for
speed.

The paper (Liu & He, arXiv:1603.01955) builds its cascaded scheme in 2-D and
names the extension to 3-D rectangular ducts as future work (Section 4); it
prints no 3-D velocity set, moment basis, duct-edge wall rule or slip
calibration.  This reference carries the 2-D method over as directly as the
definitions allow; every point below is a reading, not a printed formula:

  * Velocity set D3Q27: e = (a, b, c) with a, b, c in {-1, 0, 1}; direction
    index i = (a + 1) + 3 (b + 1) + 9 (c + 1) (rest population i = 13).
  * Collision (the 2-D collision of Eqs. 6-9 as read in clb_ref: central
    moments of the pre-collision populations about the velocity of Eq. 13,
    u = (sum e f + rho F/2) / rho, relaxed towards the central moments of the
    equilibrium): central moment k_pqr = sum_i f_i (e_x - u_x)^p
    (e_y - u_y)^q (e_z - u_z)^r, p, q, r in {0, 1, 2}; equilibrium values
    rho c_p c_q c_r with c_0 = 1, c_1 = 0, c_2 = 1/3 (the 2-D ones are
    rho c_p c_q); first order from -rho F/2 to +rho F/2 (Eq. 9's source);
    second order: trace k_200 + k_020 + k_002 towards rho at the bulk rate
    s_b (the paper's s3), its deviator and k_110, k_101, k_011 towards 0 at
    s_nu (Eq. 18); all seven third-order moments towards 0 at s_q (Eq. 21);
    every moment of order four to six at s8.
  * Rates: Eqs. (18) and (21) with N = H = ny, the duct height (Kn is the
    Knudsen number of the height); r from Eq. (21), the same on every wall.
  * Walls: half-way planes below row y = 0 and above y = ny - 1 and, for a
    duct, below layer z = 0 and above z = nz - 1 (or z periodic: a channel).
    x is periodic (force-driven, Section 3.1) or, for a pressure-driven duct
    (Section 3.2 carried to 3-D), bounded by ghost planes x = -1 and x = nx
    (below).  Eq. (20) in 3-D: when the
    pull source n - e of direction e at node n lies behind the wall planes of
    a set S of axes (one axis, or both y and z at a duct edge),
        pre_e(n) = r P_{-e}(n) + (1 - r) P_{e'}(n - e_t),
    where e' is e with its components along S reversed (specular reflection)
    and e_t is e with its components along S removed (the reflected particle
    arrives displaced along the wall by the tangential part of its path);
    with cbbsr_shift = 0 the specular source is the node n itself.  For a
    2-D slice this is exactly the rule the 2-D reference uses.  At the edges
    of a duct only the displaced source conserves mass (the same-node source
    reflects a population leaving across one wall into a direction that
    crosses both), so ducts take cbbsr_shift = 1; the same-node variant is
    kept for z-periodic channels.
  * Pressure-driven ducts: the 2-D inlet/outlet reading applied row by row
    of each cross-section: for every (y, z) the ghost population is
    f^eq(2 rho_b - rho_1, 2 u_1 - u_2) + f_1 - f^eq(rho_1, u_1), rho_1, u_1
    from the column next to the plane and u_2 from the one after it
    (rho_b = p_ratio rho_out at the inlet, rho_out at the outlet), no force;
    a pull or specular source beyond x = 0 or x = nx - 1 takes the ghost
    value.  The local Knudsen number of column x is Kn_out rho_out /
    rho_c(x), rho_c the mean pre-collision density of the central node(s) of
    the cross-section (the middle row, or the mean of the two middle rows,
    of the middle layer(s)) at the same step; s_nu(x) and s_q(x) follow from
    Eqs. (18) and (21) with N = ny; the bulk rate stays s_b.  The start is
    f^eq(rho(x), 0) with rho falling linearly from rho_in at the inlet plane
    to rho_out at the outlet (x_i = i + 1/2, L = nx).

Parity with the paper: unpinned (no 3-D scheme or number is printed).  The
reference is pinned instead by mathematics (tests/test_oracle_3d.py):
conservation, the relaxed central moments, the closed-form D3Q27
equilibrium as a fixed point, the single-rate (BGK) reduction, reduction to
the pinned 2-D reference on z-uniform states, y-z symmetry of square ducts,
the discrete slip channel of the 2-D analysis, and the continuum Poiseuille
flow rate of a rectangular duct.
"""
import dataclasses
from typing import Optional

import numpy as np

from .clb_ref import bounce_fraction, rate_nu, rate_q, slip_A1
from .rng import uniform01

# ---------------------------------------------------------------------------
# Velocity set and moment exponents.
# ---------------------------------------------------------------------------
E3 = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)], dtype=np.int64)
Q3 = 27
OPP = np.array([int(np.flatnonzero((E3 == -e).all(axis=1))[0]) for e in E3], dtype=np.int64)
REST = 13


def direction(a, b, c):
    return (a + 1) + 3 * (b + 1) + 9 * (c + 1)


# moment k = p + 3 q + 9 r  <->  exponents (p, q, r)
PQR = np.array([(p, q, r) for r in range(3) for q in range(3) for p in range(3)], dtype=np.int64)
ORDER = PQR.sum(axis=1)
C_EQ = np.array([1.0, 0.0, 1.0 / 3.0])


def moment_index(p, q, r):
    return p + 3 * q + 9 * r


@dataclasses.dataclass
class Params3D:
    nx: int
    ny: int
    nz: int
    zbc: str = "walls"            # "walls" (rectangular duct) or "periodic" (channel)
    kn: float = 0.1
    a: float = 2.0                # Bosanquet factor, Eq. (16)
    sigma: float = 1.0            # TMAC
    A1: Optional[float] = None    # B1 sigma_v; None -> from sigma
    A2: float = 0.55              # B2
    r: Optional[float] = None     # bounce-back fraction; None -> Eq. (21)
    s_b: float = 1.1              # bulk rate (the paper's s3)
    s8: float = 1.2               # rate of orders 4-6 (the paper's s8)
    gx: float = 0.0               # body acceleration
    gy: float = 0.0
    gz: float = 0.0
    rho0: float = 1.0
    tq_den: float = 16.0          # Eq. (21) denominator
    cbbsr_shift: int = 1
    xbc: str = "periodic"         # "periodic" (force-driven) or "pressure" (Section 3.2 carried to 3-D)
    p_ratio: float = 2.0          # p_in / p_out (pressure mode)
    rho_out: float = 1.0


def resolved(prm):
    A1 = prm.A1 if prm.A1 is not None else slip_A1(prm.sigma)
    r = prm.r if prm.r is not None else bounce_fraction(A1)
    return A1, r


def rho_in(prm):
    return prm.p_ratio * prm.rho_out


def rates(prm):
    """(s_b, s_nu, s_q, s8) with Eqs. (18), (21) for N = ny."""
    return (prm.s_b, rate_nu(prm.kn, prm.ny, prm.a), rate_q(prm.kn, prm.ny, prm.a, prm.A2, prm.tq_den),
            prm.s8)


# ---------------------------------------------------------------------------
# Central moments by their definition, and back.
# ---------------------------------------------------------------------------
def central_matrix(u):
    """C[n, k, i] = (e_x,i - u_x)^p (e_y,i - u_y)^q (e_z,i - u_z)^r for
    moment k = (p, q, r) and direction i, at each of the n velocities u (3, n)."""
    d = E3.T[:, None, :].astype(np.float64) - u[:, :, None]        # (3, n, 27)
    out = np.ones((u.shape[1], Q3, Q3))
    for k, (p, q, r) in enumerate(PQR):
        out[:, k, :] = d[0] ** p * d[1] ** q * d[2] ** r
    return out


def macroscopic(f, g=(0.0, 0.0, 0.0)):
    """rho and u = (sum e f + rho g / 2) / rho (Eqs. 12-13) of populations
    f (27, ...)."""
    shape = f.shape[1:]
    ff = f.reshape(Q3, -1)
    rho = ff.sum(axis=0)
    j = E3.T.astype(np.float64) @ ff
    u = j / rho + 0.5 * np.asarray(g, dtype=np.float64)[:, None]
    return rho.reshape(shape), u.reshape((3,) + shape)


def equilibrium(rho, u):
    """Populations whose central moments about u are those of the
    equilibrium, rho c_p c_q c_r: solved from the definition."""
    rho = np.atleast_1d(rho).astype(np.float64)
    u = np.asarray(u, dtype=np.float64).reshape(3, -1)
    kap = rho[None, :] * np.array([C_EQ[p] * C_EQ[q] * C_EQ[r] for p, q, r in PQR])[:, None]
    C = central_matrix(u)
    return np.linalg.solve(C, kap.T[:, :, None])[:, :, 0].T


def collide(pre, g, s_b, s_nu, s_q, s8):
    """Post-collision populations of pre (27, ...): central moments about u
    relaxed as listed in the module docstring."""
    shape = pre.shape
    f = pre.reshape(Q3, -1)
    n = f.shape[1]
    g = np.asarray(g, dtype=np.float64)
    rho = f.sum(axis=0)
    u = (E3.T.astype(np.float64) @ f) / rho + 0.5 * g[:, None]
    C = central_matrix(u)
    kap = np.einsum("nki,in->kn", C, f)
    post = np.empty_like(kap)
    k = moment_index
    # order 0 and 1
    post[k(0, 0, 0)] = kap[k(0, 0, 0)]
    post[k(1, 0, 0)] = kap[k(1, 0, 0)] + rho * g[0]
    post[k(0, 1, 0)] = kap[k(0, 1, 0)] + rho * g[1]
    post[k(0, 0, 1)] = kap[k(0, 0, 1)] + rho * g[2]
    # order 2: trace at s_b towards rho, deviator at s_nu towards 0
    diag = [k(2, 0, 0), k(0, 2, 0), k(0, 0, 2)]
    tr = kap[diag].sum(axis=0)
    tr_post = tr - s_b * (tr - rho)
    for d in diag:
        post[d] = tr_post / 3.0 + (1.0 - s_nu) * (kap[d] - tr / 3.0)
    for m in (k(1, 1, 0), k(1, 0, 1), k(0, 1, 1)):
        post[m] = (1.0 - s_nu) * kap[m]
    # orders 3 to 6
    for m in range(Q3):
        if ORDER[m] >= 3:
            s = s_q if ORDER[m] == 3 else s8
            p, q, r = PQR[m]
            eq = rho * C_EQ[p] * C_EQ[q] * C_EQ[r]
            post[m] = kap[m] - s * (kap[m] - eq)
    assert n == post.shape[1]
    out = np.linalg.solve(C, post.T[:, :, None])[:, :, 0].T
    return out.reshape(shape)


# ---------------------------------------------------------------------------
# Streaming (Eq. 5) with the walls (Eq. 20 in 3-D) -> pre-collision state.
# ---------------------------------------------------------------------------
def ghost_planes(P, prm):
    """Ghost planes x = -1 (inlet) and x = nx (outlet) of a pressure-driven
    duct, (27, nz, ny) each, by the reading in the module docstring."""
    def plane(c1, c2, rho_b):
        f1, f2 = P[:, :, :, c1], P[:, :, :, c2]
        rho1, u1 = macroscopic(f1)
        _, u2 = macroscopic(f2)
        n = rho1.size
        eq_g = equilibrium((2.0 * rho_b - rho1).ravel(), (2.0 * u1 - u2).reshape(3, n)).reshape(f1.shape)
        eq_1 = equilibrium(rho1.ravel(), u1.reshape(3, n)).reshape(f1.shape)
        return eq_g + (f1 - eq_1)
    nx = P.shape[3]
    return plane(0, 1, rho_in(prm)), plane(nx - 1, nx - 2, prm.rho_out)


def stream_bc(P, prm, r=None):
    if r is None:
        r = resolved(prm)[1]
    _, nz, ny, nx = P.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    zwalls = prm.zbc == "walls"
    pressure = prm.xbc == "pressure"
    if pressure:
        # x index shifted by one: 0 is the inlet ghost plane, nx + 1 the outlet one
        g_in, g_out = ghost_planes(P, prm)
        P = np.concatenate([g_in[..., None], P, g_out[..., None]], axis=3)
        x = x + 1
    pre = np.empty((Q3, nz, ny, nx))
    for i, (a, b, c) in enumerate(E3):
        xs = x - a if pressure else (x - a) % nx
        ys = y - b
        zs = z - c
        out_y = (ys < 0) | (ys >= ny)
        if zwalls:
            out_z = (zs < 0) | (zs >= nz)
        else:
            zs = zs % nz
            out_z = np.zeros_like(out_y)
        inside = ~out_y & ~out_z
        pre[i][inside] = P[i, zs[inside], ys[inside], xs[inside]]
        wall = ~inside
        if not wall.any():
            continue
        # reflected direction e' and the source node of its specular part
        bb = P[OPP[i], z[wall], y[wall], x[wall]]
        oy, oz = out_y[wall], out_z[wall]
        b2 = np.where(oy, -b, b)
        c2 = np.where(oz, -c, c)
        i2 = (a + 1) + 3 * (b2 + 1) + 9 * (c2 + 1)
        if prm.cbbsr_shift:
            sx = xs[wall]
            sy = np.where(oy, y[wall], ys[wall])
            sz = np.where(oz, z[wall], zs[wall])
        else:
            sx, sy, sz = x[wall], y[wall], z[wall]
        spec = P[i2, sz, sy, sx]
        pre[i][wall] = r * bb + (1.0 - r) * spec
    return pre


def central(n):
    """Index of the middle row (odd n) or of the two middle rows (even n)."""
    return [n // 2] if n % 2 else [n // 2 - 1, n // 2]


def centre_density(rho):
    """rho_c(x): mean density of the central node(s) of each cross-section,
    rho of shape (nz, ny, nx)."""
    nz, ny, _ = rho.shape
    return rho[central(nz)][:, central(ny)].mean(axis=(0, 1))


def local_rates(pre, prm):
    """s_nu(x), s_q(x) of a pressure-driven duct from the local Knudsen
    number Kn_out rho_out / rho_c(x) of the pre-collision state (Eqs. 18, 21,
    N = ny)."""
    rho, _ = macroscopic(pre)
    kn = prm.kn * prm.rho_out / centre_density(rho)
    return rate_nu(kn, prm.ny, prm.a), rate_q(kn, prm.ny, prm.a, prm.A2, prm.tq_den)


def step(P, prm):
    _, r = resolved(prm)
    pre = stream_bc(P, prm, r)
    if prm.xbc == "pressure":
        s_nu, s_q = local_rates(pre, prm)
        shape = (prm.nz, prm.ny, prm.nx)
        return collide(pre, (0.0, 0.0, 0.0), prm.s_b, np.broadcast_to(s_nu, shape).ravel(),
                       np.broadcast_to(s_q, shape).ravel(), prm.s8)
    return collide(pre, (prm.gx, prm.gy, prm.gz), *rates(prm))


def run(P, prm, nsteps):
    for _ in range(nsteps):
        P = step(P, prm)
    return P


# ---------------------------------------------------------------------------
# Initial states and diagnostics.
# ---------------------------------------------------------------------------
def init_uniform(prm):
    n = prm.nx * prm.ny * prm.nz
    feq = equilibrium(np.full(n, prm.rho0), np.zeros((3, n)))
    return feq.reshape(Q3, prm.nz, prm.ny, prm.nx)


def init_linear_rho(prm):
    """f^eq(rho(x), 0), rho falling linearly from rho_in at the inlet plane
    x = 0 to rho_out at the outlet plane x = nx (node centres x_i = i + 1/2)."""
    x = np.arange(prm.nx, dtype=np.float64) + 0.5
    rho = rho_in(prm) - (rho_in(prm) - prm.rho_out) * x / prm.nx
    rho3 = np.broadcast_to(rho, (prm.nz, prm.ny, prm.nx)).ravel()
    n = rho3.size
    return equilibrium(rho3, np.zeros((3, n))).reshape(Q3, prm.nz, prm.ny, prm.nx)


def init_perturbed(prm, seed, amp):
    """P_i = f_i^eq(rho0, 0) + amp (2U - 1), U from SplitMix64 keyed by
    seed XOR (27 * node + i), node = (z * ny + y) * nx + x."""
    P = init_uniform(prm)
    node = np.arange(prm.nz * prm.ny * prm.nx, dtype=np.uint64).reshape(prm.nz, prm.ny, prm.nx)
    for i in range(Q3):
        U = uniform01(seed, np.uint64(27) * node + np.uint64(i))
        P[i] += amp * (2.0 * U - 1.0)
    return P


def init_perturbed_window(prm, seed, amp, y0, y1, z0, z1):
    """Rows y0 .. y1 - 1 of layers z0 .. z1 - 1 (full width) of
    init_perturbed: the same generator keyed by the same node numbers,
    evaluated for that window only (ducts too large to hold whole)."""
    P = init_uniform(dataclasses.replace(prm, ny=y1 - y0, nz=z1 - z0))
    zz = np.arange(z0, z1, dtype=np.uint64)[:, None, None]
    yy = np.arange(y0, y1, dtype=np.uint64)[None, :, None]
    xx = np.arange(prm.nx, dtype=np.uint64)[None, None, :]
    node = (zz * np.uint64(prm.ny) + yy) * np.uint64(prm.nx) + xx
    for i in range(Q3):
        U = uniform01(seed, np.uint64(27) * node + np.uint64(i))
        P[i] += amp * (2.0 * U - 1.0)
    return P


def run_window(P, prm, nsteps):
    """nsteps steps of a window of full-width rows P (27, layers, rows, nx)
    cut out of the duct prm: the rates of Eqs. (18), (21) use the duct's
    N = prm.ny, and every face of the window is stepped as a wall (Eq. 20 in
    3-D).  Where the window ends at a duct wall that is the duct's own rule;
    at a cut face it is not, and after nsteps the rows and layers within
    nsteps of a cut face no longer hold the duct's values (the others do).
    A z-periodic channel keeps its periodic z only in a window of all its
    layers."""
    _, r = resolved(prm)
    zbc = prm.zbc if P.shape[1] == prm.nz else "walls"
    win = dataclasses.replace(prm, ny=P.shape[2], nz=P.shape[1], zbc=zbc)
    rt = rates(prm)
    g = (prm.gx, prm.gy, prm.gz)
    for _ in range(nsteps):
        P = collide(stream_bc(P, win, r), g, *rt)
    return P


def moments(P, prm):
    """rho (nz, ny, nx) and u (3, nz, ny, nx) of the pre-collision state."""
    return macroscopic(stream_bc(P, prm), (prm.gx, prm.gy, prm.gz))


def mass_flow(P, prm):
    """m(x) = sum_{y,z} rho u_x of the pre-collision state (a pressure-driven
    duct's mass flow through each cross-section)."""
    rho, u = moments(P, prm)
    return (rho * u[0]).sum(axis=(0, 1))


def pressure_deviation(P, prm):
    """delta p(x) = (p_c(x) - p_l(x)) / p_out along the duct's centre line,
    p = rho/3, p_l linear from p_in at x = 0 to p_out at x = L = nx."""
    rho, _ = moments(P, prm)
    p_out, p_in = prm.rho_out / 3.0, rho_in(prm) / 3.0
    x = np.arange(prm.nx, dtype=np.float64) + 0.5
    p_l = p_in - (p_in - p_out) * x / prm.nx
    return (centre_density(rho) / 3.0 - p_l) / p_out


def flow_rate_Q(P, prm):
    """Dimensionless flow rate of Section 3.1 carried over to a duct of
    height H = ny and width W = nz: Q = sqrt(6) sum_{y,z} u_x / (3 g H^2 W),
    averaged over x (for a z-periodic channel the 2-D Q)."""
    _, u = moments(P, prm)
    H, W = float(prm.ny), float(prm.nz)
    return u[0].sum(axis=(0, 1)).mean() * np.sqrt(6.0) / (3.0 * prm.gx * H * H * W)
