"""D2Q9 lattice algebra for the CLB oracle (test infrastructure only).

Everything here is built from the definitions in Section 2.1 of the paper:
the velocity set of Eq. (1), the orthogonal collision basis K of Eq. (3)
(from its column definitions), the raw-moment matrix T of Eq. (10) (from its
row definitions) and the equilibrium moments of Eq. (11).  T is inverted in
exact rational arithmetic.  The shift from raw to central moments is the
binomial expansion the paper invokes after Eq. (8).
"""
from fractions import Fraction
from math import comb, cos, sin, pi, sqrt

import numpy as np

# --------------------------------------------------------------------------
# Eq. (1): e_0 = (0,0); e_i = (cos((i-1)pi/2), sin((i-1)pi/2)) for i = 1..4;
# e_i = sqrt(2) (cos((2i-9)pi/4), sin((2i-9)pi/4)) for i = 5..8; c = 1.
# --------------------------------------------------------------------------
def _velocities():
    out = [(0, 0)]
    for i in range(1, 5):
        ang = (i - 1) * pi / 2
        out.append((round(cos(ang)), round(sin(ang))))
    for i in range(5, 9):
        ang = (2 * i - 9) * pi / 4
        out.append((round(sqrt(2) * cos(ang)), round(sqrt(2) * sin(ang))))
    return out


E = np.array(_velocities(), dtype=np.int64)          # (9, 2)
EX = E[:, 0]
EY = E[:, 1]
Q = 9


def _vec(fn):
    return np.array([fn(int(ex), int(ey)) for ex, ey in E], dtype=np.int64)


# --------------------------------------------------------------------------
# Eq. (3): K = [|1>, |ex>, |ey>, 3|ex^2+ey^2> - 4|1>, |ex^2-ey^2>, |ex ey>,
#               -3|ex^2 ey> + 2|ey>, -3|ex ey^2> + 2|ex>,
#               9|ex^2 ey^2> - 6|ex^2+ey^2> + 4|1>]   (columns)
# --------------------------------------------------------------------------
K_COLUMNS = [
    lambda x, y: 1,
    lambda x, y: x,
    lambda x, y: y,
    lambda x, y: 3 * (x * x + y * y) - 4,
    lambda x, y: x * x - y * y,
    lambda x, y: x * y,
    lambda x, y: -3 * x * x * y + 2 * y,
    lambda x, y: -3 * x * y * y + 2 * x,
    lambda x, y: 9 * x * x * y * y - 6 * (x * x + y * y) + 4,
]
K = np.stack([_vec(c) for c in K_COLUMNS], axis=1)   # (9, 9), K[i, k]

# --------------------------------------------------------------------------
# Eq. (10): T = [|1>, |ex>, |ey>, |ex^2+ey^2>, |ex^2-ey^2>, |ex ey>,
#                |ex^2 ey>, |ex ey^2>, |ex^2 ey^2>]^T   (rows)
# --------------------------------------------------------------------------
T_ROWS = [
    lambda x, y: 1,
    lambda x, y: x,
    lambda x, y: y,
    lambda x, y: x * x + y * y,
    lambda x, y: x * x - y * y,
    lambda x, y: x * y,
    lambda x, y: x * x * y,
    lambda x, y: x * y * y,
    lambda x, y: x * x * y * y,
]
T = np.stack([_vec(r) for r in T_ROWS], axis=0)       # (9, 9), T[k, i]


def exact_inverse(mat):
    """Gauss-Jordan inverse of an integer matrix in exact rationals."""
    n = len(mat)
    a = [[Fraction(int(mat[i][j])) for j in range(n)] +
         [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        p = a[col][col]
        a[col] = [v / p for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                fac = a[r][col]
                a[r] = [vr - fac * vc for vr, vc in zip(a[r], a[col])]
    return [row[n:] for row in a]


T_INV_EXACT = exact_inverse(T)                        # list of lists of Fraction
T_INV = np.array([[float(v) for v in row] for row in T_INV_EXACT])

# --------------------------------------------------------------------------
# Raw -> central moment shift (text after Eq. 8: central moments are binomial
# combinations of raw moments).  Work in the monomial basis
#   (1, x, y, xx, yy, xy, xxy, xyy, xxyy)  ->  exponents (a, b)
# where  kappa_ab = sum_{p<=a, q<=b} C(a,p) C(b,q) (-ux)^(a-p) (-uy)^(b-q) m_pq,
# then change to the T basis of Eq. (10), whose rows 3 and 4 are xx+yy and
# xx-yy.
# --------------------------------------------------------------------------
MONOMIALS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
# B maps monomial-basis moments to T-basis moments.
B = np.zeros((9, 9), dtype=np.int64)
B[0, 0] = 1
B[1, 1] = 1
B[2, 2] = 1
B[3, 3] = 1; B[3, 4] = 1      # xx + yy
B[4, 3] = 1; B[4, 4] = -1     # xx - yy
B[5, 5] = 1
B[6, 6] = 1
B[7, 7] = 1
B[8, 8] = 1
B_INV = np.array([[float(v) for v in row] for row in exact_inverse(B)])


def monomial_shift(ux, uy):
    """(n, 9, 9) matrices taking raw monomial moments to central ones about u."""
    ux = np.asarray(ux)
    uy = np.asarray(uy)
    n = ux.shape[0]
    dtype = np.result_type(ux.dtype, uy.dtype, np.float64)
    S = np.zeros((n, 9, 9), dtype=dtype)
    for r, (a, b) in enumerate(MONOMIALS):
        for c, (p, q) in enumerate(MONOMIALS):
            if p <= a and q <= b:
                S[:, r, c] = comb(a, p) * comb(b, q) * (-ux) ** (a - p) * (-uy) ** (b - q)
    return S


def central_shift(ux, uy):
    """N(u): (n, 9, 9) matrices taking T-basis raw moments to T-basis central
    moments about u.  N(u)^-1 = N(-u)."""
    S = monomial_shift(ux, uy)
    return np.matmul(np.matmul(B.astype(np.float64), S), B_INV)


# --------------------------------------------------------------------------
# Eq. (11): T-basis raw moments of the equilibrium; f_eq = T^-1 f_eq_hat.
# --------------------------------------------------------------------------
def feq_hat(rho, ux, uy):
    rho = np.asarray(rho)
    return np.stack([
        rho,
        rho * ux,
        rho * uy,
        2.0 / 3.0 * rho + rho * (ux * ux + uy * uy),
        rho * (ux * ux - uy * uy),
        rho * ux * uy,
        rho * uy / 3.0 + rho * ux * ux * uy,
        rho * ux / 3.0 + rho * ux * uy * uy,
        rho / 9.0 + rho * (ux * ux + uy * uy) / 3.0 + rho * ux * ux * uy * uy,
    ])


def feq(rho, ux, uy):
    """Equilibrium populations f_i^eq, shape (9,) + rho.shape."""
    fh = feq_hat(rho, ux, uy)
    flat = fh.reshape(9, -1)
    return (T_INV @ flat).reshape(fh.shape)
