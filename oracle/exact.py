"""Exact rational evaluation of the CLB step, node by node (test infrastructure).

Independent of the vectorised reference in ``clb_ref``: it follows the printed
closed form of the collision (Eqs. 6-9, with S = T^-1 S_hat where T^-1 is the
exact rational inverse of Eq. 10) and performs streaming (Eq. 5) and the CBBSR
walls (Eq. 20) by looking up each neighbour explicitly.  All arithmetic is in
fractions.Fraction, so the result has no rounding at all; comparing the FP64
reference with it bounds the reference's error and catches formula mistakes
that happen to be self-consistent in floating point.
"""
from fractions import Fraction

from .lattice import E, K, T_INV_EXACT

F0 = Fraction(0)


def _frac(v):
    return v if isinstance(v, Fraction) else Fraction(v)


def collide_node(f, Fx, Fy, s3, s4, s5, s6, s7, s8):
    """Post-collision populations of one node, Eqs. (6)-(9), exact."""
    f = [_frac(v) for v in f]
    Fx, Fy = _frac(Fx), _frac(Fy)
    s3, s4, s5, s6, s7, s8 = (_frac(v) for v in (s3, s4, s5, s6, s7, s8))
    half = Fraction(1, 2)
    # Eq. (8): raw moments <ex^m ey^n | f> from the velocity set itself.
    def mom(m, n):
        return sum((f[i] * (int(E[i][0]) ** m) * (int(E[i][1]) ** n) for i in range(9)), F0)
    rho = mom(0, 0)
    kx, ky = mom(1, 0), mom(0, 1)
    kxx, kyy, kxy = mom(2, 0), mom(0, 2), mom(1, 1)
    kxxy, kxyy, kxxyy = mom(2, 1), mom(1, 2), mom(2, 2)
    # Eq. (13)
    ux = kx / rho + half * Fx
    uy = ky / rho + half * Fy
    # Eq. (7)
    g3 = s3 / 12 * (Fraction(2, 3) * rho + rho * (ux * ux + uy * uy) - (kxx + kyy)
                    - half * rho * (2 * Fx * ux + 2 * Fy * uy))
    g4 = s4 / 4 * (rho * (ux * ux - uy * uy) - (kxx - kyy)
                   - half * rho * (2 * Fx * ux - 2 * Fy * uy))
    g5 = s5 / 4 * (rho * ux * uy - kxy - half * rho * (Fx * uy + Fy * ux))
    g6 = (s6 / 4 * (2 * rho * ux * ux * uy + kxxy - 2 * ux * kxy - uy * kxx
                    - half * rho * (Fy * ux * ux + 2 * Fx * ux * uy))
          - half * uy * (3 * g3 + g4) - 2 * ux * g5)
    g7 = (s7 / 4 * (2 * rho * ux * uy * uy + kxyy - 2 * uy * kxy - ux * kyy
                    - half * rho * (Fx * uy * uy + 2 * Fy * uy * ux))
          - half * ux * (3 * g3 - g4) - 2 * uy * g5)
    g8 = (s8 / 4 * (rho / 9 + 3 * rho * ux * ux * uy * uy
                    - (kxxyy - 2 * ux * kxyy - 2 * uy * kxxy + ux * ux * kyy
                       + uy * uy * kxx + 4 * ux * uy * kxy)
                    - half * rho * (2 * Fx * ux * uy * uy + 2 * Fy * uy * ux * ux))
          - 2 * g3 - half * uy * uy * (3 * g3 + g4) - half * ux * ux * (3 * g3 - g4)
          - 4 * ux * uy * g5 - 2 * uy * g6 - 2 * ux * g7)
    # Eq. (9)
    S_hat = [F0, rho * Fx, rho * Fy, 2 * rho * (ux * Fx + uy * Fy),
             2 * rho * (ux * Fx - uy * Fy), rho * (ux * Fy + uy * Fx),
             rho * Fy * ux * ux + 2 * rho * Fx * ux * uy,
             rho * Fx * uy * uy + 2 * rho * Fy * uy * ux,
             2 * rho * Fx * ux * uy * uy + 2 * rho * Fy * uy * ux * ux]
    S = [sum((T_INV_EXACT[i][k] * S_hat[k] for k in range(9)), F0) for i in range(9)]
    g = [F0, F0, F0, g3, g4, g5, g6, g7, g8]
    # Eq. (6), written as f + K g + S with K from its column definitions (Eq. 3).
    return [f[i] + sum((int(K[i][k]) * g[k] for k in range(9)), F0) + S[i] for i in range(9)]


def gather_node(P, nx, ny, x, y, r, shift=True):
    """Pre-collision populations of node (x, y) on a periodic-x channel with
    CBBSR walls below row 0 and above row ny-1.  P[i][y][x] nested lists."""
    r = _frac(r)
    out = [None] * 9
    for i in range(9):
        sx = (x - int(E[i][0])) % nx
        sy = y - int(E[i][1])
        if 0 <= sy < ny:
            out[i] = P[i][sy][sx]
    xm, xp = (x - 1) % nx, (x + 1) % nx
    if y == 0:
        out[2] = P[4][0][x]
        out[5] = r * P[7][0][x] + (1 - r) * P[8][0][xm if shift else x]
        out[6] = r * P[8][0][x] + (1 - r) * P[7][0][xp if shift else x]
    if y == ny - 1:
        t = ny - 1
        out[4] = P[2][t][x]
        out[7] = r * P[5][t][x] + (1 - r) * P[6][t][xp if shift else x]
        out[8] = r * P[6][t][x] + (1 - r) * P[5][t][xm if shift else x]
    return out


def step_grid(P, nx, ny, r, Fx, Fy, s3, s_nu, s_q, s8, shift=True):
    """One exact step of a periodic-x channel; P as nested lists [i][y][x]."""
    new = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    for y in range(ny):
        for x in range(nx):
            pre = gather_node(P, nx, ny, x, y, r, shift)
            post = collide_node(pre, Fx, Fy, s3, s_nu, s_nu, s_q, s_q, s8)
            for i in range(9):
                new[i][y][x] = post[i]
    return new
