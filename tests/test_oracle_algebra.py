"""Pins of the CPU reference's single-node algebra against what the paper fixes.

Section 2.1 of Liu & He (arXiv:1603.01955): Eq. (3) K, Eqs. (6)-(9) closed-form
collision, Eq. (10) T, Eq. (11) equilibrium, Eqs. (12)-(13) macroscopics.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from clb_inputs import uniform_populations
from oracle import clb_ref as C
from oracle import exact as X
from oracle import lattice as L

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(v) for v in line.split()])
    return np.array(rows, dtype=np.int64)


def _rand_nodes(n, seed):
    return uniform_populations(n, 1, seed)[:, 0, :]          # (9, n)


def _exact_central(f, ux, uy, a, b):
    return sum((f[i] * (int(L.E[i][0]) - ux) ** a * (int(L.E[i][1]) - uy) ** b
                for i in range(9)), Fraction(0))


def _exact_feq(rho, ux, uy):
    fh = [rho, rho * ux, rho * uy,
          Fraction(2, 3) * rho + rho * (ux * ux + uy * uy), rho * (ux * ux - uy * uy),
          rho * ux * uy, rho * uy / 3 + rho * ux * ux * uy, rho * ux / 3 + rho * ux * uy * uy,
          rho / 9 + rho * (ux * ux + uy * uy) / 3 + rho * ux * ux * uy * uy]
    return [sum((L.T_INV_EXACT[i][k] * fh[k] for k in range(9)), Fraction(0)) for i in range(9)]


# P1: the printed matrices equal their column / row definitions.
def test_K_matches_printed_eq3():
    assert np.array_equal(L.K, _load_matrix("K_eq3.txt"))
    # K is orthogonal: its columns are mutually orthogonal.
    G = L.K.T @ L.K
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0


def test_T_matches_printed_eq10():
    assert np.array_equal(L.T, _load_matrix("T_eq10.txt"))


def test_T_inverse_exact():
    prod = [[sum((L.T_INV_EXACT[i][k] * int(L.T[k][j]) for k in range(9)), Fraction(0))
             for j in range(9)] for i in range(9)]
    assert all(prod[i][j] == (1 if i == j else 0) for i in range(9) for j in range(9))
    # Only denominators 1, 2, 4 occur, so the FP64 copy is exact.
    assert {v.denominator for row in L.T_INV_EXACT for v in row} <= {1, 2, 4}


def test_velocity_set_eq1():
    speeds = (L.EX ** 2 + L.EY ** 2)
    assert speeds.tolist() == [0, 1, 1, 1, 1, 2, 2, 2, 2]
    # opposite pairs
    for i, j in [(1, 3), (2, 4), (5, 7), (6, 8)]:
        assert (L.E[i] == -L.E[j]).all()


# P2: the expanded updates of Eq. (6) are K g.
def test_eq6_rows_are_K_times_g():
    assert np.array_equal(_load_matrix("eq6_coefficients.txt"), L.K)


# P3: closed form (Eqs. 6-9) == explicit-matrix central-moment relaxation.
@pytest.mark.parametrize("F", [(0.0, 0.0), (1e-3, -2e-3), (0.05, 0.02)])
def test_closed_form_equals_matrix_form_fp64(F):
    f = _rand_nodes(400, 11)
    rates = (1.1, 0.37, 0.37, 0.81, 0.81, 1.2)
    a = C.collide(f, F[0], F[1], rates[0], rates[1], rates[3], rates[5])
    b = C.collide_literal(f, F[0], F[1], *rates)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(f))


def test_matrix_form_vs_exact_rationals():
    f = _rand_nodes(25, 12)
    Fx, Fy = 3e-3, -1e-3
    s = (1.1, 0.6, 0.6, 0.9, 0.9, 1.2)
    got = C.collide(f, Fx, Fy, s[0], s[1], s[3], s[5])
    for n in range(f.shape[1]):
        ref = X.collide_node([Fraction(v) for v in f[:, n]], Fraction(Fx), Fraction(Fy),
                             *[Fraction(v) for v in s])
        ref = np.array([float(v) for v in ref])
        assert np.max(np.abs(got[:, n] - ref)) <= 1e-15 * 8


def test_closed_form_relaxes_central_moments_exactly():
    """Exact rationals: after the collision of Eqs. (6)-(9) the central moments
    about the physical velocity of Eq. (13) are relaxed individually towards
    those of the equilibrium (Eq. 11) -- the defining property of the cascaded
    operator (Section 2.1) -- and the first-order ones flip from -rho F/2 to
    +rho F/2."""
    f_all = _rand_nodes(6, 13)
    Fx, Fy = Fraction(1, 250), Fraction(-3, 1000)
    s = dict(s3=Fraction(11, 10), s4=Fraction(3, 7), s5=Fraction(3, 7),
             s6=Fraction(5, 6), s7=Fraction(5, 6), s8=Fraction(6, 5))
    for n in range(f_all.shape[1]):
        f = [Fraction(v) for v in f_all[:, n]]
        post = X.collide_node(f, Fx, Fy, **s)
        rho = sum(f)
        ux = sum(f[i] * int(L.E[i][0]) for i in range(9)) / rho + Fx / 2
        uy = sum(f[i] * int(L.E[i][1]) for i in range(9)) / rho + Fy / 2
        c = lambda g, a, b: _exact_central(g, ux, uy, a, b)
        assert c(f, 1, 0) == -rho * Fx / 2 and c(post, 1, 0) == rho * Fx / 2
        assert c(f, 0, 1) == -rho * Fy / 2 and c(post, 0, 1) == rho * Fy / 2
        tr = lambda g: c(g, 2, 0) + c(g, 0, 2)
        df = lambda g: c(g, 2, 0) - c(g, 0, 2)
        assert tr(post) == tr(f) - s["s3"] * (tr(f) - Fraction(2, 3) * rho)
        assert df(post) == df(f) - s["s4"] * df(f)
        assert c(post, 1, 1) == c(f, 1, 1) - s["s5"] * c(f, 1, 1)
        assert c(post, 2, 1) == c(f, 2, 1) - s["s6"] * c(f, 2, 1)
        assert c(post, 1, 2) == c(f, 1, 2) - s["s7"] * c(f, 1, 2)
        assert c(post, 2, 2) == c(f, 2, 2) - s["s8"] * (c(f, 2, 2) - rho / 9)


# P4: mass conserved exactly; momentum gains exactly rho F.
def test_conservation_exact():
    f_all = _rand_nodes(5, 14)
    Fx, Fy = Fraction(1, 100), Fraction(1, 300)
    for n in range(5):
        f = [Fraction(v) for v in f_all[:, n]]
        post = X.collide_node(f, Fx, Fy, Fraction(11, 10), Fraction(1, 3), Fraction(1, 3),
                              Fraction(1, 2), Fraction(1, 2), Fraction(6, 5))
        rho = sum(f)
        assert sum(post) == rho
        jx = lambda g: sum(g[i] * int(L.E[i][0]) for i in range(9))
        jy = lambda g: sum(g[i] * int(L.E[i][1]) for i in range(9))
        assert jx(post) == jx(f) + rho * Fx
        assert jy(post) == jy(f) + rho * Fy


def test_conservation_fp64_matrix_form():
    f = _rand_nodes(1000, 15)
    post = C.collide(f, 2e-3, 1e-3, 1.1, 0.2, 0.3, 1.2)
    rho = f.sum(0)
    assert np.max(np.abs(post.sum(0) - rho)) <= 1e-15 * 16
    jx = lambda g: np.tensordot(L.EX.astype(float), g, (0, 0))
    assert np.max(np.abs(jx(post) - jx(f) - rho * 2e-3)) <= 1e-15 * 16


# P5: the forcing S = T^-1 S_hat (Eq. 9) has first-order central moments rho F
# and no central moments of order two or more.
def test_forcing_central_moments_exact():
    f_all = _rand_nodes(4, 16)
    Fx, Fy = Fraction(7, 1000), Fraction(-2, 1000)
    zero = Fraction(0)
    for n in range(4):
        f = [Fraction(v) for v in f_all[:, n]]
        S = [p - q for p, q in zip(X.collide_node(f, Fx, Fy, zero, zero, zero, zero, zero, zero), f)]
        rho = sum(f)
        ux = sum(f[i] * int(L.E[i][0]) for i in range(9)) / rho + Fx / 2
        uy = sum(f[i] * int(L.E[i][1]) for i in range(9)) / rho + Fy / 2
        assert sum(S) == 0
        assert _exact_central(S, ux, uy, 1, 0) == rho * Fx
        assert _exact_central(S, ux, uy, 0, 1) == rho * Fy
        for a, b in [(2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]:
            assert _exact_central(S, ux, uy, a, b) == 0


# P6: the equilibrium at rest is the textbook D2Q9 weight set (4/9, 1/9, 1/36)
# of Qian et al. (1992), the lattice the paper uses; any equilibrium is a fixed
# point of the force-free collision.
def test_equilibrium_at_rest_is_d2q9_weights():
    w = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    rho = Fraction(13, 10)
    assert _exact_feq(rho, Fraction(0), Fraction(0)) == [rho * v for v in w]
    assert np.allclose(C.init_uniform(C.Params(nx=1, ny=1))[:, 0, 0], [float(v) for v in w],
                       rtol=0, atol=2e-16)


def test_equilibrium_is_fixed_point():
    rng = np.random.default_rng(17)
    rho = rng.uniform(0.8, 1.2, 50)
    ux = rng.uniform(-0.1, 0.1, 50)
    uy = rng.uniform(-0.1, 0.1, 50)
    f = L.feq(rho, ux, uy)
    post = C.collide(f, 0.0, 0.0, 1.1, 0.3, 0.7, 1.2)
    assert np.max(np.abs(post - f)) <= 1e-15 * 4
    # exact version
    fe = _exact_feq(Fraction(11, 10), Fraction(1, 20), Fraction(-1, 30))
    assert X.collide_node(fe, 0, 0, Fraction(11, 10), Fraction(1, 3), Fraction(1, 3),
                          Fraction(1, 2), Fraction(1, 2), Fraction(6, 5)) == fe


# P7: equal rates reduce the cascaded operator to BGK with forcing:
# post = (1 - s) f + s f_eq(rho, u) + (1 - s/2) S; s = 1, F = 0 gives f_eq.
def test_equal_rates_reduce_to_bgk_exact():
    f_all = _rand_nodes(3, 18)
    Fx, Fy = Fraction(1, 200), Fraction(1, 500)
    s = Fraction(7, 10)
    zero = Fraction(0)
    for n in range(3):
        f = [Fraction(v) for v in f_all[:, n]]
        post = X.collide_node(f, Fx, Fy, s, s, s, s, s, s)
        S = [p - q for p, q in zip(X.collide_node(f, Fx, Fy, zero, zero, zero, zero, zero, zero), f)]
        rho = sum(f)
        ux = sum(f[i] * int(L.E[i][0]) for i in range(9)) / rho + Fx / 2
        uy = sum(f[i] * int(L.E[i][1]) for i in range(9)) / rho + Fy / 2
        fe = _exact_feq(rho, ux, uy)
        bgk = [(1 - s) * f[i] + s * fe[i] + (1 - s / 2) * S[i] for i in range(9)]
        assert post == bgk
        one = Fraction(1)
        rho0 = sum(f)
        u0x = sum(f[i] * int(L.E[i][0]) for i in range(9)) / rho0
        u0y = sum(f[i] * int(L.E[i][1]) for i in range(9)) / rho0
        assert X.collide_node(f, 0, 0, one, one, one, one, one, one) == _exact_feq(rho0, u0x, u0y)
