"""Pressure-driven long channel (Section 3.2 of Liu & He, arXiv:1603.01955):
pins of the CPU reference by internal invariants and the lubrication limit.

The paper delegates the inlet/outlet treatment to an external reference whose
details it does not print, so the ghost-column reading used here has no
number in the paper to match: parity against the paper is unpinned; these
tests pin what any correct pressure-driven steady state must satisfy.
"""
import numpy as np
import pytest

from oracle import analytic as A
from oracle import clb_ref as C


@pytest.fixture(scope="module")
def steady_long_channel():
    prm = C.Params(nx=100, ny=6, xbc="pressure", kn=0.1, p_ratio=2.0)
    P = C.init_linear_rho(prm)
    for _ in range(20):
        P = C.run(P, prm, 500)
        m = C.column_sums(P, prm)[0]
        if (m.max() - m.min()) / m.mean() < 1e-7:
            break
    return prm, P


def test_mass_flow_uniform_along_channel(steady_long_channel):
    prm, P = steady_long_channel
    m = C.column_sums(P, prm)[0]
    assert (m.max() - m.min()) / m.mean() < 1e-6


def test_mirror_symmetry_about_centreline(steady_long_channel):
    prm, P = steady_long_channel
    _, ux, uy = C.moments(P, prm)
    assert np.max(np.abs(ux - ux[::-1])) <= 1e-14 * np.max(np.abs(ux))
    assert np.max(np.abs(uy + uy[::-1])) <= 1e-14 * np.max(np.abs(ux))


def test_pressure_deviation_bulge_and_lubrication(steady_long_channel):
    """Compressible flow: the centre-line pressure lies above the linear
    profile (positive deviation, Figs. 3-5 of the paper); mass flow and
    deviation follow the lubrication model to a few per cent."""
    prm, P = steady_long_channel
    dp = C.pressure_deviation(P, prm)
    assert dp[5:-5].min() > 0
    A1, _ = C.resolved(prm)
    m_lub, p_lub = A.lubrication_profile(prm.nx, prm.ny, prm.kn, prm.p_ratio, prm.a, A1, prm.A2)
    m = C.column_sums(P, prm)[0].mean()
    assert abs(m / m_lub - 1) < 0.03
    p_out = 1.0 / 3.0
    x = C.x_positions(prm)
    dp_lub = (np.array(p_lub) - (2 * p_out - p_out * x / prm.nx)) / p_out
    assert abs(dp.max() / dp_lub.max() - 1) < 0.06


def test_slip_grows_downstream(steady_long_channel):
    """Section 3.2: the slip velocity increases along the channel as the
    pressure (and the local Kn) falls."""
    prm, P = steady_long_channel
    _, ux, _ = C.moments(P, prm)
    slip = ux[0] / ux.max(axis=0)
    assert slip[-10] > slip[10]


@pytest.mark.parametrize("nx,ny,kn,ratio", [(2000, 20, 0.1, 1.8), (400, 7, 0.47, 2.0), (100, 40, 0.01, 1.2)])
def test_noslip_massflow_integrates_the_lubrication_equation(nx, ny, kn, ratio):
    """The closed-form m_ns equals the lubrication equation integrated
    numerically (RK4 from the outlet, m by bisection on the inlet pressure)
    with every rarefaction term switched off: no slip (A1 = A2 = 0), no
    Bosanquet factor (a = 0), no discrete wall term."""
    m_num, _ = A.lubrication_profile(nx, ny, kn, ratio, 0.0, 0.0, 0.0, nsub=4, discrete=False)
    assert abs(A.noslip_massflow(nx, ny, kn, ratio) / m_num - 1.0) <= 1e-9


def test_noslip_massflow_is_poiseuille_at_mean_density():
    """p_in^2 - p_out^2 = 2 p_mean (p_in - p_out), so the compressible m_ns is
    plane Poiseuille flow, m = rho H^3 (p_in - p_out) / (12 mu L), with rho the
    mean of the inlet and outlet densities, at any pressure ratio."""
    nx, ny, kn, rho_out = 500, 16, 0.2, 1.3
    for ratio in (1.001, 1.8, 3.0):
        m = A.noslip_massflow(nx, ny, kn, ratio, rho_out=rho_out)
        rho = rho_out * (1.0 + ratio) / 2.0
        mu = np.sqrt(6.0 / np.pi) * rho_out * kn * ny / 3.0
        dp = (ratio - 1.0) * rho_out / 3.0
        assert abs(m / (rho * ny ** 3 * dp / (12.0 * mu * nx)) - 1.0) <= 1e-12


def test_slip_raises_the_lubrication_mass_flow_above_noslip():
    """With slip and the Bosanquet factor the lubrication model carries more
    mass than the no-slip channel, more so at larger Kn_out (S > 1 and
    increasing; at ratio 1.8, sigma = 0.93 as in the paper's mass-flow study)."""
    A1 = C.slip_A1(0.93)
    S = [A.lubrication_profile(200, 10, kn, 1.8, 2.0, A1, 0.55, nsub=2)[0] / A.noslip_massflow(200, 10, kn, 1.8)
         for kn in (0.02, 0.1, 0.4)]
    assert 1.0 < S[0] < S[1] < S[2]


def test_pressure_driven_channel_carries_the_eq19_slip():
    """Without a body force the steady pressure-driven channel carries the
    mass flow of the lubrication model built on the slip law of Eq. (19)
    itself (second-order coefficient 12 B2), not the force-driven periodic
    channel's discrete 18 B2: at Kn_out = 0.5 (200 x 4, ratio 1.8,
    sigma = 0.93) the two models differ by 6%."""
    prm = C.Params(nx=200, ny=4, xbc="pressure", kn=0.5, p_ratio=1.8, sigma=0.93)
    P = C.init_linear_rho(prm)
    prev = None
    for _ in range(60):
        P = C.run(P, prm, 500)
        m = C.column_sums(P, prm)[0].mean()
        if prev is not None and abs(m - prev) <= 1e-7 * abs(m):
            break
        prev = m
    A1, _ = C.resolved(prm)
    m12, _ = A.lubrication_profile(200, 4, 0.5, 1.8, 2.0, A1, 0.55, nsub=2, c2=12.0)
    m18, _ = A.lubrication_profile(200, 4, 0.5, 1.8, 2.0, A1, 0.55, nsub=2, c2=18.0)
    assert abs(m / m12 - 1.0) < 0.01
    assert m / m18 < 0.95


@pytest.mark.parametrize("ny", [5, 6])
def test_local_knudsen_number_follows_the_centre_line(ny):
    """Section 3.2: the local Kn scales inversely with the centre-line
    pressure.  A column whose centre-line density is k rho_out relaxes with
    the rates a periodic channel of Kn = Kn_out / k has, whatever the density
    of the rows off the centre line."""
    prm = C.Params(nx=4, ny=ny, xbc="pressure", kn=0.3, p_ratio=1.5, rho_out=1.1)
    ks = np.array([0.7, 1.0, 1.3, 2.1])
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.5, 2.0, size=(ny, 4))        # off-centre rows: anything
    mid = [ny // 2] if ny % 2 else [ny // 2 - 1, ny // 2]
    if ny % 2:
        rho[mid[0]] = ks * prm.rho_out
    else:                                            # the mean of the two middle rows counts
        rho[mid[0]] = ks * prm.rho_out * 0.8
        rho[mid[1]] = ks * prm.rho_out * 1.2
    pre = np.stack([w * rho for w in (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)])
    s_nu, s_q = C.step_rates(pre, prm)
    for x, k in enumerate(ks):
        per = C.Params(nx=4, ny=ny, kn=prm.kn / k)
        nu_ref, q_ref = C.step_rates(pre, per)
        assert abs(s_nu[x] - nu_ref) <= 1e-15 and abs(s_q[x] - q_ref) <= 1e-15
    # changing only off-centre rows leaves the rates alone
    rho2 = rho.copy()
    off = [y for y in range(ny) if y not in mid]
    rho2[off] *= 1.7
    pre2 = np.stack([w * rho2 for w in (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)])
    s_nu2, s_q2 = C.step_rates(pre2, prm)
    assert np.array_equal(s_nu, s_nu2) and np.array_equal(s_q, s_q2)


@pytest.mark.parametrize("ny", [4, 5])
def test_linear_rest_state_has_no_pressure_deviation(ny):
    """Closed-form special case: at rest with the density linear between
    rho_in on the inlet plane and rho_out on the outlet plane, streaming keeps
    every column's density (the ghost columns continue the line), so the
    centre-line pressure is the linear profile itself: delta p(x) = 0 at
    every column, the edge columns included.  The pull of Eq. (5) gives the
    pre-collision state the momentum -(1/3) d rho/dx away from the walls,
    the same in every column, and so the mass flow m(x) is uniform."""
    prm = C.Params(nx=10, ny=ny, xbc="pressure", kn=0.2, p_ratio=1.7, rho_out=1.2)
    P = C.init_linear_rho(prm)
    rho0 = P.sum(0)[0]
    x = np.arange(10) + 0.5                          # node centres; planes at 0 and 10
    assert np.allclose(rho0, 1.7 * 1.2 + (1.2 - 1.7 * 1.2) * x / 10, rtol=0, atol=1e-15)
    dp = C.pressure_deviation(P, prm)
    assert np.max(np.abs(dp)) <= 1e-14
    rho, ux, _ = C.moments(P, prm)
    slope = (1.2 - 1.7 * 1.2) / 10
    assert np.allclose((rho * ux)[1:-1], -slope / 3, rtol=0, atol=1e-15)
    m = C.column_sums(P, prm)[0]
    assert m.min() > 0 and np.max(np.abs(m - m[0])) <= 1e-14
