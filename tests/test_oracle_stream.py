"""Pins of the CPU reference's streaming and boundaries (Eqs. 5 and 20,
Sections 3.1-3.2 of Liu & He, arXiv:1603.01955)."""
from fractions import Fraction

import numpy as np
import pytest

from clb_inputs import uniform_populations
from oracle import clb_ref as C
from oracle import exact as X
from oracle import lattice as L


def _jx(f):
    return np.tensordot(L.EX.astype(float), f, (0, 0))


@pytest.mark.parametrize("shift", [1, 0])
@pytest.mark.parametrize("shape", [(7, 5), (1, 3), (4, 1), (1, 1)])
def test_stream_conserves_mass(shift, shape):
    """P8: streaming with CBBSR walls (weights r, 1-r sum to one) and
    periodic x moves mass without creating or losing any."""
    nx, ny = shape
    P = uniform_populations(nx, ny, 21)
    prm = C.Params(nx=nx, ny=ny, cbbsr_shift=shift, r=0.37)
    pre = C.stream_bc(P, prm)
    assert abs(pre.sum() - P.sum()) <= 1e-14 * P.sum()


@pytest.mark.parametrize("shift", [1, 0])
def test_gather_nodes_matches_stream(shift):
    P = uniform_populations(6, 5, 22)
    prm = C.Params(nx=6, ny=5, cbbsr_shift=shift, r=0.41)
    pre = C.stream_bc(P, prm)
    ys, xs = np.meshgrid(np.arange(5), np.arange(6), indexing="ij")
    got = C.gather_nodes(P, prm, ys.ravel(), xs.ravel())
    assert np.array_equal(got, pre.reshape(9, -1))


def test_specular_walls_conserve_x_momentum():
    """P9: with r = 0 the walls reflect specularly, so they exert no shear:
    the total x-momentum grows by exactly g * total mass per step."""
    prm = C.Params(nx=5, ny=6, r=0.0, gx=1e-3, kn=0.3)
    P = uniform_populations(5, 6, 23)
    for _ in range(4):
        pre = C.stream_bc(P, prm)
        assert abs(_jx(pre).sum() - _jx(P).sum()) <= 1e-14
        Pn = C.step(P, prm)
        assert abs(_jx(Pn).sum() - _jx(P).sum() - prm.gx * P.sum()) <= 1e-14
        P = Pn


def test_bounce_back_reverses_wall_momentum():
    """P9: with r = 1 the wall returns every outgoing particle reversed, so the
    wall rows gain no net tangential momentum from streaming across the wall."""
    prm = C.Params(nx=4, ny=3, r=1.0)
    P = uniform_populations(4, 3, 24)
    pre = C.stream_bc(P, prm)
    # bottom row: what arrives in 2, 5, 6 is what left in 4, 7, 8 at the same node
    np.testing.assert_array_equal(pre[[2, 5, 6], 0], P[[4, 7, 8], 0])
    np.testing.assert_array_equal(pre[[4, 7, 8], 2], P[[2, 5, 6], 2])


def test_x_translation_invariance():
    prm = C.Params(nx=7, ny=4, gx=1e-3, kn=0.5)
    P = uniform_populations(7, 4, 25)
    a = np.roll(C.run(P, prm, 3), 2, axis=2)
    b = C.run(np.roll(P, 2, axis=2), prm, 3)
    assert np.max(np.abs(a - b)) <= 1e-15


def test_mirror_symmetry():
    """P10: for a y-mirror-symmetric start (2<->4, 5<->8, 6<->7, y -> ny-1-y)
    and a force along x, the state stays mirror-symmetric."""
    prm = C.Params(nx=3, ny=6, gx=1e-4, kn=0.2)
    P = uniform_populations(3, 6, 26)
    mirror = [0, 1, 4, 3, 2, 8, 7, 6, 5]
    P = 0.5 * (P + P[mirror][:, ::-1, :])
    for _ in range(5):
        P = C.step(P, prm)
        assert np.max(np.abs(P - P[mirror][:, ::-1, :])) <= 1e-15
    rho, ux, uy = C.moments(P, prm)
    assert np.max(np.abs(ux - ux[::-1])) <= 1e-15
    assert np.max(np.abs(uy + uy[::-1])) <= 1e-15


@pytest.mark.parametrize("shift", [True, False])
def test_brute_force_exact_tiny_grid(shift):
    """P17: two steps on a 4x3 channel: FP64 reference vs node-by-node exact
    rational evaluation of Eqs. (5), (6)-(9) and (20)."""
    nx, ny = 4, 3
    P0 = uniform_populations(nx, ny, 27)
    r = Fraction(5, 8)
    Fx, Fy = Fraction(1, 1000), Fraction(-1, 4000)
    s3, snu, sq, s8 = Fraction(11, 10), Fraction(2, 5), Fraction(3, 4), Fraction(6, 5)
    # The FP64 reference with the same (rational, exactly representable) rates.
    prm = C.Params(nx=nx, ny=ny, r=float(r), gx=float(Fx), gy=float(Fy), cbbsr_shift=int(shift))
    P = P0.copy()
    Pe = [[[Fraction(v) for v in row] for row in plane] for plane in P0]
    for _ in range(2):
        pre = C.stream_bc(P, prm)
        P = C.collide(pre, prm.gx, prm.gy, float(s3), float(snu), float(sq), float(s8))
        Pe = X.step_grid(Pe, nx, ny, r, Fx, Fy, s3, snu, sq, s8, shift)
    ref = np.array([[[float(v) for v in row] for row in plane] for plane in Pe])
    assert np.max(np.abs(P - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_pressure_rest_state_is_steady():
    """Equal inlet and outlet pressure: the uniform rest state is a fixed
    point of the whole step including the ghost columns."""
    prm = C.Params(nx=6, ny=4, xbc="pressure", kn=0.2, p_ratio=1.0, rho_out=1.0)
    P = C.init_linear_rho(prm)
    Pn = C.run(P, prm, 3)
    assert np.max(np.abs(Pn - P)) <= 1e-15


def test_pressure_ghost_density_is_linear():
    """Ghost columns place the prescribed density on the inlet/outlet planes:
    (rho_ghost + rho_adjacent)/2 = rho_boundary."""
    prm = C.Params(nx=5, ny=3, xbc="pressure", kn=0.2, p_ratio=1.7, rho_out=1.0)
    P = uniform_populations(5, 3, 28)
    g_in, g_out = C.ghost_columns(P, prm)
    assert np.allclose(0.5 * (g_in.sum(0) + P[:, :, 0].sum(0)), 1.7, rtol=0, atol=1e-15)
    assert np.allclose(0.5 * (g_out.sum(0) + P[:, :, -1].sum(0)), 1.0, rtol=0, atol=1e-15)


def _second_moments(f):
    """Pxx, Pyy, Pxy of populations f (9, ny), straight from Eq. (1)'s velocities."""
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)[:, None]
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)[:, None]
    return (ex * ex * f).sum(0), (ey * ey * f).sum(0), (ex * ey * f).sum(0)


def test_pressure_ghost_velocity_is_extrapolated():
    """The ghost column's velocity (its own first moments over its density)
    continues the two adjacent columns linearly: u_g = 2 u_1 - u_2.  The
    copied non-equilibrium part carries no mass or momentum, so this holds
    for an arbitrary state."""
    prm = C.Params(nx=6, ny=4, xbc="pressure", kn=0.2, p_ratio=1.6, rho_out=1.1)
    P = uniform_populations(6, 4, 29, lo=0.05, hi=0.2)
    g_in, g_out = C.ghost_columns(P, prm)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)[:, None]
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)[:, None]

    def vel(f):
        return (ex * f).sum(0) / f.sum(0), (ey * f).sum(0) / f.sum(0)
    for g, c1, c2 in ((g_in, 0, 1), (g_out, -1, -2)):
        ug, vg = vel(g)
        u1, v1 = vel(P[:, :, c1])
        u2, v2 = vel(P[:, :, c2])
        assert np.allclose(ug, 2 * u1 - u2, rtol=0, atol=1e-14)
        assert np.allclose(vg, 2 * v1 - v2, rtol=0, atol=1e-14)


def test_pressure_ghost_copies_the_nonequilibrium_stress():
    """The ghost column keeps the adjacent column's non-equilibrium part: its
    second moments minus those of the D2Q9 equilibrium at its own density
    and velocity (rho/3 + rho u u, from Eq. 11's moments) equal the same
    difference for the adjacent column; an equilibrium neighbour gives an
    equilibrium ghost."""
    prm = C.Params(nx=5, ny=3, xbc="pressure", kn=0.2, p_ratio=1.8, rho_out=1.0)
    P = uniform_populations(5, 3, 30, lo=0.05, hi=0.2)
    g_in, g_out = C.ghost_columns(P, prm)

    def neq_stress(f):
        rho = f.sum(0)
        ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)[:, None]
        ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)[:, None]
        u, v = (ex * f).sum(0) / rho, (ey * f).sum(0) / rho
        pxx, pyy, pxy = _second_moments(f)
        return pxx - (rho / 3 + rho * u * u), pyy - (rho / 3 + rho * v * v), pxy - rho * u * v
    for g, c1 in ((g_in, 0), (g_out, -1)):
        for a, b in zip(neq_stress(g), neq_stress(P[:, :, c1])):
            assert np.allclose(a, b, rtol=0, atol=1e-14)
    # equilibrium neighbours: the ghost is itself an equilibrium (no stress left)
    Q = C.init_linear_rho(prm)
    g_in, g_out = C.ghost_columns(Q, prm)
    for g in (g_in, g_out):
        for a in neq_stress(g):
            assert np.max(np.abs(a)) <= 1e-15


def test_perturbed_start_counter_layout():
    """The seeded start depends only on (seed, node, direction)."""
    prm = C.Params(nx=5, ny=3)
    a = C.init_perturbed(prm, 99, 1e-4)
    big = C.init_perturbed(C.Params(nx=5, ny=6), 99, 1e-4)
    assert np.array_equal(a, big[:, :3, :])
    w = C.init_uniform(prm)
    assert np.max(np.abs(a - w)) <= 1e-4 and np.max(np.abs(a - w)) > 5e-5


def test_perturbed_rows_are_rows_of_the_start():
    """init_perturbed_rows gives exactly the rows of the whole seeded start."""
    prm = C.Params(nx=9, ny=11)
    whole = C.init_perturbed(prm, 1234, 1e-3)
    for y0, y1 in ((0, 4), (3, 10), (8, 11), (5, 6)):
        assert np.array_equal(C.init_perturbed_rows(prm, 1234, 1e-3, y0, y1), whole[:, y0:y1])


@pytest.mark.parametrize("shift", [1, 0])
def test_row_bands_reproduce_the_channel(shift):
    """Bands of rows stepped on their own (rates from the channel's height)
    equal the whole channel's run on every row more than n steps away from a
    cut edge: the band reaching each wall, and interior bands."""
    nx, ny, n = 13, 17, 3
    prm = C.Params(nx=nx, ny=ny, kn=0.7, gx=2e-4, gy=-3e-5, cbbsr_shift=shift, forcing=1)
    P0 = C.init_perturbed(prm, 77, 1e-3)
    whole = C.run(P0, prm, n)
    # bottom band: rows 0 .. 2n, valid rows 0 .. n
    got = C.run_rows(P0[:, :2 * n + 1].copy(), prm, n)
    assert np.array_equal(got[:, :n + 1], whole[:, :n + 1])
    # top band: rows ny - 2n - 1 .. ny - 1, valid rows ny - n - 1 .. ny - 1
    got = C.run_rows(P0[:, ny - 2 * n - 1:].copy(), prm, n)
    assert np.array_equal(got[:, n:], whole[:, ny - n - 1:])
    # interior bands: only the middle row is valid
    for yc in (n, 8, ny - n - 1):
        got = C.run_rows(P0[:, yc - n:yc + n + 1].copy(), prm, n)
        assert np.array_equal(got[:, n], whole[:, yc])
    # and a cut row is not the channel's (the band edges are not walls there)
    got = C.run_rows(P0[:, 8 - n:8 + n + 1].copy(), prm, n)
    assert not np.array_equal(got[:, 0], whole[:, 8 - n])
