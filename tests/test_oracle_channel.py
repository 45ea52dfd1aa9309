"""Pins of the CPU reference against closed-form steady channel flows and the
numbers printed in Section 3.1 of Liu & He (arXiv:1603.01955)."""
import os
from math import pi, sqrt

import numpy as np
import pytest

from oracle import analytic as A
from oracle import clb_ref as C
from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_values():
    out = {}
    with open(os.path.join(GOLDEN, "paper_values.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def _steady(prm, max_steps=60000, check=500, tol=1e-13):
    P = C.init_uniform(prm)
    prev = None
    for n in range(0, max_steps, check):
        P = C.run(P, prm, check)
        su = C.column_sums(P, prm)[1].mean()
        if prev is not None and abs(su - prev) <= tol * abs(su):
            return P, n + check
        prev = su
    return P, max_steps


def test_splitmix64_published_outputs():
    """SplitMix64 seeded with 0: first three outputs of the public reference code."""
    keys = np.array([0, int(rng.GAMMA), (2 * int(rng.GAMMA)) % 2 ** 64], dtype=np.uint64)
    got = [int(v) for v in rng.splitmix64_first(keys)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_section3_parameters():
    pv = _paper_values()
    # sigma = 1: B1 = 1 - 0.1817 = 0.8183, sigma_v = 1.
    assert abs(C.slip_A1(1.0) - (1 - pv["slip_B1_coeff"])) < 1e-15
    # Fig. 1 Knudsen numbers Kn = 2k/sqrt(pi) quoted in the text.
    assert round(2 * pv["fig1_k_min"] / sqrt(pi), 4) == pv["fig1_kn_first"]
    assert round(2 * pv["fig1_k_max"] / sqrt(pi), 4) == pv["fig1_kn_last"]


# A1 = B1 sigma_v with B1 = 1 - 0.1817 sigma (Section 3) and
# sigma_v = (2 - sigma)/sigma (Section 2.3), worked out by hand as exact
# fractions, e.g. sigma = 0.93: (0.831019 x 1.07)/0.93 = 88919033/93000000;
# r = 1/(1 + A1 sqrt(pi/6)) (Eq. 21) to 12 digits.
SLIP_LITERALS = [
    # sigma, A1, r
    (0.93, 0.956118634408602, 0.591069422151),   # the mass-flow study's TMAC (Section 3.2)
    (0.7, 1.62093285714286, 0.460212543396),
    (1.5, 0.242483333333333, 0.850729877251),
]


@pytest.mark.parametrize("sigma,A1,r", SLIP_LITERALS)
def test_slip_coefficients_away_from_full_accommodation(sigma, A1, r):
    """At sigma = 1 both sigma_v = 1 and B1 = 0.8183 hide a wrong sigma
    dependence; these TMACs do not."""
    assert abs(C.slip_A1(sigma) - A1) <= 1e-13
    assert abs(C.bounce_fraction(C.slip_A1(sigma)) - r) <= 1e-11
    prm = C.Params(nx=1, ny=8, sigma=sigma)
    got_A1, got_r = C.resolved(prm)
    assert abs(got_A1 - A1) <= 1e-13 and abs(got_r - r) <= 1e-11


@pytest.mark.parametrize("ny,kn", [(16, 0.1), (12, 0.5)])
def test_continuum_slip_at_tmac_093(ny, kn):
    """With sigma = 0.93 and 24 in Eq. (21), the steady force-driven channel
    of the reference carries the continuum slip law of Eq. (19): its
    sum_y u_x equals the second-order slip Poiseuille flow whose A1 = B1
    sigma_v is written out here from sigma, not taken from the reference."""
    sigma = 0.93
    A1 = (1.0 - 0.1817 * sigma) * ((2.0 - sigma) / sigma)
    prm = C.Params(nx=1, ny=ny, kn=kn, gx=1e-6, sigma=sigma, tq_den=24.0)
    P, _ = _steady(prm)
    _, ux, _ = C.moments(P, prm)
    cont = A.continuum_sum_u(ny, kn, 2.0, A1, 0.55, 1e-6)
    assert abs(ux[:, 0].sum() / cont - 1) <= 1e-6


@pytest.fixture(scope="module")
def channel_4x32():
    """Force-driven periodic channel 4 x 32, Kn = 0.1, g = 1e-6, 20,000 steps."""
    prm = C.Params(nx=4, ny=32, kn=0.1, gx=1e-6)
    return prm, C.run(C.init_uniform(prm), prm, 20000)


def test_discrete_closed_form_channel(channel_4x32):
    """P11: the steady x-uniform solution of the scheme is the discrete
    slip-parabola u = U_s + G y (H - y); nonlinear terms are O(u^2) ~ 1e-8."""
    prm, P = channel_4x32
    _, r = C.resolved(prm)
    _, ux, uy = C.moments(P, prm)
    Us, G, rows, su = A.discrete_channel(32, 0.1, 2.0, 0.55, r, 1e-6)
    for x in range(4):
        assert np.max(np.abs(ux[:, x] - rows) / np.array(rows)) <= 1e-6
    assert abs(ux[:, 0].sum() / su - 1) <= 1e-6
    assert np.max(np.abs(uy)) <= 1e-14
    # flow rate of Section 3.1
    assert abs(C.flow_rate_Q(P, prm) / A.discrete_Q(32, 0.1, 2.0, 0.55, r) - 1) <= 1e-6


def test_excess_over_continuum_second_order_slip(channel_4x32):
    """P12: with the printed Eq. (21) the scheme's flow exceeds the continuum
    second-order slip profile (Eq. 19) by 3g/(16 tt) + (pi/4) B2 tt g per row."""
    prm, P = channel_4x32
    A1, _ = C.resolved(prm)
    _, ux, _ = C.moments(P, prm)
    cont = A.continuum_sum_u(32, 0.1, 2.0, A1, 0.55, 1e-6)
    tt = C.tau_tilde(0.1, 32, 2.0)
    excess = 32 * (3e-6 / (16 * tt) + pi / 4 * 0.55 * tt * 1e-6)
    assert abs(ux[:, 0].sum() - cont - excess) <= 1e-6 * cont
    assert 0.0160 < ux[:, 0].sum() / cont - 1 < 0.0165


def test_denominator_24_matches_continuum_slip():
    """P12: with 24 in place of 16 in Eq. (21) the scheme reproduces the
    continuum second-order slip profile of Eq. (19)."""
    prm = C.Params(nx=1, ny=16, kn=0.1, gx=1e-6, tq_den=24.0)
    P, _ = _steady(prm)
    A1, _ = C.resolved(prm)
    _, ux, _ = C.moments(P, prm)
    cont = A.continuum_sum_u(16, 0.1, 2.0, A1, 0.55, 1e-6)
    assert abs(ux[:, 0].sum() / cont - 1) <= 1e-6


@pytest.mark.parametrize("ny,kn", [(16, 0.1), (16, 1.0), (8, 0.3)])
def test_third_order_forcing_gives_continuum_slip_with_printed_denominator(ny, kn):
    """With the source's third-order moments of a second-order (Guo-type)
    force term, (1 - s_q/2) rho F/3 in k_xyy, the printed Eq. (21) (16)
    reproduces the continuum second-order slip profile of Eq. (19): the
    force-driven excess of Eq. (9)'s source (+1.6% at H = 32) vanishes."""
    prm = C.Params(nx=1, ny=ny, kn=kn, gx=1e-6, forcing=1)
    P, _ = _steady(prm)
    A1, _ = C.resolved(prm)
    _, ux, _ = C.moments(P, prm)
    cont = A.continuum_sum_u(ny, kn, 2.0, A1, 0.55, 1e-6)
    assert abs(ux[:, 0].sum() / cont - 1) <= 1e-8


def test_third_order_forcing_changes_only_third_moments():
    """The variant keeps mass and momentum of every node and differs from the
    Eq. (9) collision only in the raw moments k_xxy, k_xyy, by
    (1 - s_q/2) rho (F_y, F_x) / 3."""
    rng_ = np.random.default_rng(5)
    f = rng_.uniform(0.05, 0.15, size=(9, 40))
    gx, gy, sq = 3e-3, -2e-3, 0.7
    a = C.collide(f, gx, gy, 1.1, 0.4, sq, 1.2)
    b = C.collide(f, gx, gy, 1.1, 0.4, sq, 1.2, forcing=1)
    d = C.T @ (b - a)
    rho = f.sum(axis=0)
    assert np.max(np.abs(d[[0, 1, 2, 3, 4, 5, 8]])) <= 1e-16
    assert np.allclose(d[6], (1 - sq / 2) * rho * gy / 3, rtol=1e-12, atol=0)
    assert np.allclose(d[7], (1 - sq / 2) * rho * gx / 3, rtol=1e-12, atol=0)


def test_no_slip_magic_combination():
    """P13: r = 1 with (tau_s - 1/2)(tau_q - 1/2) = 1/8 (B2 = 0, denominator
    24) gives the exact no-slip Poiseuille parabola."""
    prm = C.Params(nx=1, ny=16, kn=0.1, gx=1e-6, r=1.0, A2=0.0, tq_den=24.0)
    P, _ = _steady(prm)
    _, ux, _ = C.moments(P, prm)
    tt = C.tau_tilde(0.1, 16, 2.0)
    y = np.arange(16) + 0.5
    ref = 1.5e-6 / tt * y * (16 - y)
    assert np.max(np.abs(ux[:, 0] - ref)) <= 1e-6 * ref.max()


@pytest.mark.parametrize("ny,kn", [(16, 0.1), (9, 0.4)])
def test_flow_rate_scale_on_the_no_slip_parabola(ny, kn):
    """The normalisation of Q (Section 3.1) on a flow known in closed form.
    Q = int u dy / (F_x H^2 sqrt(RT/2) / p) with F_x = rho0 g, RT = 1/3 and
    p = rho0/3 is sqrt(6) int u dy / (3 g H^2).  With r = 1 and the magic
    combination the steady profile is the no-slip parabola u = g y (H - y)/(2 nu)
    with nu = tt/3 (Eq. 14) and tt = sqrt(6/pi) H k_e, k_e = Kn/(1 + a Kn)
    (Eqs. 15-18).  Its midpoint sum over the H rows at y = j + 1/2 is
    (g/(2 nu)) (H^3/6 + H/12), so Q = (sqrt(pi)/(12 k_e)) (1 + 1/(2 H^2))."""
    a = 2.0
    prm = C.Params(nx=1, ny=ny, kn=kn, a=a, gx=1e-6, r=1.0, A2=0.0, tq_den=24.0)
    P, _ = _steady(prm)
    ke = kn / (1.0 + a * kn)
    ref = sqrt(pi) / (12.0 * ke) * (1.0 + 1.0 / (2.0 * ny * ny))
    assert abs(C.flow_rate_Q(P, prm) / ref - 1) <= 1e-6


@pytest.mark.parametrize("kn", [0.3, 0.87, 3.0])
def test_flow_rate_matches_discrete_closed_form(kn):
    """P14: converged Q of the reference equals the discrete closed form."""
    prm = C.Params(nx=1, ny=16, kn=kn, gx=1e-6)
    P, _ = _steady(prm)
    _, r = C.resolved(prm)
    assert abs(C.flow_rate_Q(P, prm) / A.discrete_Q(16, kn, 2.0, 0.55, r) - 1) <= 1e-6


def test_knudsen_minimum_location():
    """P14: the scheme's flow rate has its minimum at Kn* = 1/(sqrt(18 B2) - a)
    = 0.872, where the paper reports a minimum near Kn = 0.9 (Abstract, Section 3.1); the
    continuum law (2 B2) would put it at 1.76."""
    pv = _paper_values()
    kstar = A.knudsen_minimum(pv["rarefaction_factor_a"], pv["slip_B2"])
    assert abs(kstar - 0.8723) < 1e-3
    assert round(kstar, 1) == pv["knudsen_minimum_clb"]
    r = C.bounce_fraction(C.slip_A1(1.0))
    grid = np.exp(np.linspace(np.log(0.1), np.log(10.0), 2001))
    for N in (16, 32, 64, 128):
        q = [A.discrete_Q(N, k, 2.0, 0.55, r) for k in grid]
        assert 0.85 < grid[int(np.argmin(q))] < 0.90
    big = [A.large_N_Q(k, 2.0, C.slip_A1(1.0), 0.55) for k in grid]
    assert abs(grid[int(np.argmin(big))] - kstar) < 5e-3
