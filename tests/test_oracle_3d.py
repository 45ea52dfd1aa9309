"""Pins of the 3-D (D3Q27) cascaded reference for rectangular microducts.

The paper gives no 3-D scheme (it names the extension as future work), so
these pins come from mathematics and from the pinned 2-D reference: exact
conservation, the closed-form D3Q27 equilibrium, the single-rate (BGK)
reduction, reduction to the 2-D step on z-uniform states, the y-z symmetry
of square ducts, the discrete slip channel of the 2-D analysis, and the
continuum Poiseuille flow rate of a rectangular duct."""
from math import pi, tanh

import dataclasses

import numpy as np
import pytest

from oracle import analytic as A
from oracle import clb3d_ref as D
from oracle import clb_ref as C
from oracle.lattice import E as E2


def _random_state(shape, seed, lo=0.02, hi=0.06):
    return np.random.default_rng(seed).uniform(lo, hi, size=(27,) + shape)


def _w(e, u):
    """Factor of the D3Q27 equilibrium along one axis: the D1Q3 populations
    with moments 1, u, 1/3 + u^2."""
    return 2.0 / 3.0 - u * u if e == 0 else 0.5 * (1.0 / 3.0 + u * u + e * u)


def _phi(e, u, k):
    """D1Q3 populations whose central moments about u are (1, 0, 0) for
    k = 0 and (0, 1, 0) for k = 1 (solved by hand from the three moment
    equations)."""
    if k == 0:
        return 1.0 - u * u if e == 0 else 0.5 * (u * u + e * u)
    return -2.0 * u if e == 0 else u + 0.5 * e


def test_velocity_set():
    assert len({tuple(e) for e in D.E3}) == 27
    assert (D.E3[D.OPP] == -D.E3).all()
    assert D.REST == D.direction(0, 0, 0) and (D.E3[D.REST] == 0).all()
    for i, (a, b, c) in enumerate(D.E3):
        assert D.direction(a, b, c) == i


def test_collision_conserves_mass_and_adds_the_force():
    f = _random_state((50,), 1)
    g = np.array([3e-3, -2e-3, 1e-3])
    out = D.collide(f, g, 1.1, 0.7, 0.9, 1.2)
    rho = f.sum(axis=0)
    assert np.max(np.abs(out.sum(axis=0) - rho)) <= 1e-15
    for ax in range(3):
        j0 = (D.E3[:, ax][:, None] * f).sum(axis=0)
        j1 = (D.E3[:, ax][:, None] * out).sum(axis=0)
        assert np.max(np.abs(j1 - (j0 + rho * g[ax]))) <= 1e-15


def test_post_collision_central_moments_are_the_relaxed_ones():
    """Central moments of the output, computed direction by direction about
    the pre-collision velocity, equal the relaxed pre-collision moments."""
    f = _random_state((20,), 2)
    g = np.array([1e-3, 2e-3, -1e-3])
    s_b, s_nu, s_q, s8 = 1.3, 0.6, 0.8, 1.1
    out = D.collide(f, g, s_b, s_nu, s_q, s8)
    rho = f.sum(axis=0)
    u = (D.E3.T @ f) / rho + 0.5 * g[:, None]

    def mom(h, p, q, r):
        e = D.E3.astype(float)
        return sum(h[i] * (e[i, 0] - u[0]) ** p * (e[i, 1] - u[1]) ** q * (e[i, 2] - u[2]) ** r
                   for i in range(27))

    for ax, pqr in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        assert np.allclose(mom(out, *pqr), rho * g[ax] / 2, rtol=0, atol=2e-15)
        assert np.allclose(mom(f, *pqr), -rho * g[ax] / 2, rtol=0, atol=2e-15)
    tr_in = mom(f, 2, 0, 0) + mom(f, 0, 2, 0) + mom(f, 0, 0, 2)
    tr_out = mom(out, 2, 0, 0) + mom(out, 0, 2, 0) + mom(out, 0, 0, 2)
    assert np.allclose(tr_out, (1 - s_b) * tr_in + s_b * rho, rtol=0, atol=2e-15)
    for pqr in [(2, 0, 0), (0, 2, 0), (0, 0, 2)]:
        dev_in, dev_out = mom(f, *pqr) - tr_in / 3, mom(out, *pqr) - tr_out / 3
        assert np.allclose(dev_out, (1 - s_nu) * dev_in, rtol=0, atol=2e-15)
    for pqr in [(1, 1, 0), (1, 0, 1), (0, 1, 1)]:
        assert np.allclose(mom(out, *pqr), (1 - s_nu) * mom(f, *pqr), rtol=0, atol=2e-15)
    ceq = {0: 1.0, 1: 0.0, 2: 1.0 / 3.0}
    for p in range(3):
        for q in range(3):
            for r in range(3):
                n = p + q + r
                if n < 3:
                    continue
                s = s_q if n == 3 else s8
                eq = rho * ceq[p] * ceq[q] * ceq[r]
                assert np.allclose(mom(out, p, q, r), (1 - s) * mom(f, p, q, r) + s * eq, rtol=0, atol=2e-15)


def test_equilibrium_is_the_product_form():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.8, 1.2, 10)
    u = rng.uniform(-0.1, 0.1, (3, 10))
    feq = D.equilibrium(rho, u)
    ref = np.array([[rho[n] * _w(a, u[0, n]) * _w(b, u[1, n]) * _w(c, u[2, n]) for n in range(10)]
                    for a, b, c in D.E3])
    assert np.max(np.abs(feq - ref)) <= 1e-15
    rest = D.equilibrium(np.array([1.0]), np.zeros((3, 1)))[:, 0]
    w0 = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for i, e in enumerate(D.E3):
        assert abs(rest[i] - w0[int(np.abs(e).sum())]) <= 1e-15


def test_equilibrium_is_a_fixed_point_for_any_rates():
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.8, 1.2, 10)
    u = rng.uniform(-0.1, 0.1, (3, 10))
    feq = D.equilibrium(rho, u)
    out = D.collide(feq, np.zeros(3), 1.7, 0.3, 1.4, 0.6)
    assert np.max(np.abs(out - feq)) <= 1e-15


def test_single_rate_reduces_to_bgk_with_the_force_source():
    """All rates s: f' = (1 - s) f + s f^eq(rho, u) + (1 - s/2) S with S the
    populations whose only nonzero central moments are the first-order rho F."""
    f = _random_state((12,), 5)
    g = np.array([2e-3, -1e-3, 5e-4])
    s = 0.8
    out = D.collide(f, g, s, s, s, s)
    rho = f.sum(axis=0)
    u = (D.E3.T @ f) / rho + 0.5 * g[:, None]
    feq = D.equilibrium(rho, u)
    S = np.zeros_like(f)
    for i, (a, b, c) in enumerate(D.E3):
        for n in range(f.shape[1]):
            px = [_phi(a, u[0, n], 1), _phi(a, u[0, n], 0)]
            py = [_phi(b, u[1, n], 1), _phi(b, u[1, n], 0)]
            pz = [_phi(c, u[2, n], 1), _phi(c, u[2, n], 0)]
            S[i, n] = rho[n] * (g[0] * px[0] * py[1] * pz[1] + g[1] * px[1] * py[0] * pz[1]
                                + g[2] * px[1] * py[1] * pz[0])
    ref = (1 - s) * f + s * feq + (1 - s / 2) * S
    assert np.max(np.abs(out - ref)) <= 1e-15


@pytest.mark.parametrize("shift", [1, 0])
def test_reduces_to_the_2d_step_on_z_uniform_states(shift):
    """z-periodic, z-uniform and z-mirror-symmetric states: summed over e_z
    the 3-D populations advance exactly as the pinned 2-D reference (with the
    bulk rate equal to s_nu, where a 2-D slice relaxes each normal stress at
    s_nu both ways)."""
    nx, ny = 7, 5
    P2 = np.random.default_rng(6).uniform(0.02, 0.06, (9, ny, nx))
    # split each D2Q9 population over e_z = -1, 0, +1 in a fixed symmetric way
    wz = {-1: 0.25, 0: 0.5, 1: 0.25}
    P3 = np.zeros((27, 3, ny, nx))
    idx2 = {(int(e[0]), int(e[1])): k for k, e in enumerate(E2)}
    for i, (a, b, c) in enumerate(D.E3):
        P3[i] = wz[int(c)] * P2[idx2[(int(a), int(b))]][None]
    kn, gx = 0.4, 1e-3
    snu = C.rate_nu(kn, ny, 2.0)
    p3 = D.Params3D(nx=nx, ny=ny, nz=3, zbc="periodic", kn=kn, gx=gx, s_b=snu, cbbsr_shift=shift)
    p2 = C.Params(nx=nx, ny=ny, kn=kn, gx=gx, s3=snu, cbbsr_shift=shift)
    for _ in range(4):
        P3 = D.step(P3, p3)
        P2 = C.step(P2, p2)
        for z in range(3):
            m = np.zeros_like(P2)
            for i, (a, b, c) in enumerate(D.E3):
                m[idx2[(int(a), int(b))]] += P3[i, z]
            assert np.max(np.abs(m - P2)) <= 1e-14


def test_square_duct_step_commutes_with_the_y_z_swap():
    n = 5
    prm = D.Params3D(nx=4, ny=n, nz=n, kn=0.3, gx=1e-3)
    P = _random_state((n, n, 4), 7)

    def swap(Q):
        out = np.empty_like(Q)
        for i, (a, b, c) in enumerate(D.E3):
            out[D.direction(a, c, b)] = np.swapaxes(Q[i], 0, 1)
        return out

    a = swap(D.step(P, prm))
    b = D.step(swap(P), prm)
    assert np.max(np.abs(a - b)) <= 1e-15


@pytest.mark.parametrize("zbc,shift,r", [("walls", 1, None), ("walls", 1, 0.3), ("periodic", 1, 0.0),
                                         ("walls", 1, 1.0), ("periodic", 0, 0.3)])
def test_streaming_with_walls_conserves_mass(zbc, shift, r):
    prm = D.Params3D(nx=3, ny=4, nz=2, zbc=zbc, cbbsr_shift=shift, r=r)
    P = _random_state((2, 4, 3), 8)
    pre = D.stream_bc(P, prm)
    assert abs(pre.sum() - P.sum()) <= 1e-14


def test_same_node_specular_source_loses_mass_at_duct_edges():
    """Taking the specular part from the node itself (cbbsr_shift = 0) is
    not conservative once two wall planes meet: a population leaving an edge
    node across one wall is reflected into a direction that crosses both, so
    no node takes it up.  Only the displaced source is used for ducts."""
    prm = D.Params3D(nx=3, ny=4, nz=2, zbc="walls", cbbsr_shift=0, r=0.3)
    P = _random_state((2, 4, 3), 8)
    assert abs(D.stream_bc(P, prm).sum() - P.sum()) > 1e-3


def test_edge_rule_at_a_duct_edge():
    """Direction (1, 1, 1) at the edge node (x, 0, 0): both walls crossed;
    bounce-back from (-1, -1, -1) at the node, specular (-y, -z reversed)
    from (1, -1, -1) one node upstream in x."""
    prm = D.Params3D(nx=4, ny=3, nz=3, r=0.4)
    P = _random_state((3, 3, 4), 9)
    pre = D.stream_bc(P, prm)
    i = D.direction(1, 1, 1)
    for x in range(4):
        want = 0.4 * P[D.direction(-1, -1, -1), 0, 0, x] + 0.6 * P[D.direction(1, -1, -1), 0, 0, (x - 1) % 4]
        assert abs(pre[i, 0, 0, x] - want) <= 1e-17
    # (1, 1, -1) at (x, 0, 0) crosses only the y wall: specular from (1, -1, -1) at (x - 1, 0, 1)
    i = D.direction(1, 1, -1)
    for x in range(4):
        want = 0.4 * P[D.direction(-1, -1, 1), 0, 0, x] + 0.6 * P[D.direction(1, -1, -1), 1, 0, (x - 1) % 4]
        assert abs(pre[i, 0, 0, x] - want) <= 1e-17


def _steady(prm, P=None, check=500, tol=1e-11, cap=60000):
    P = D.init_uniform(prm) if P is None else P
    prev = None
    for n in range(0, cap, check):
        P = D.run(P, prm, check)
        q = D.flow_rate_Q(P, prm)
        if prev is not None and abs(q - prev) <= tol * abs(q):
            return P
        prev = q
    raise AssertionError("no steady state")


def test_channel_is_the_discrete_slip_channel():
    """A z-periodic force-driven 3-D channel carries the steady profile of
    the 2-D discrete analysis (parabola plus the slip of Eqs. 20-21),
    whatever the bulk rate."""
    ny, kn, g = 12, 0.2, 1e-6
    prm = D.Params3D(nx=1, ny=ny, nz=1, zbc="periodic", kn=kn, gx=g)
    P = _steady(prm)
    _, u = D.moments(P, prm)
    _, r = D.resolved(prm)
    _, _, rows, _ = A.discrete_channel(ny, kn, 2.0, 0.55, r, g)
    assert np.max(np.abs(u[0, 0, :, 0] / np.array(rows) - 1)) <= 1e-6
    assert np.max(np.abs(u[1])) <= 1e-13 and np.max(np.abs(u[2])) <= 1e-13


def _duct_mean_velocity(H, W, g, nu, terms=200):
    """Continuum no-slip Poiseuille flow in an H x W rectangle (H <= W):
    mean velocity g H^2 / (12 nu) [1 - (192 H / (pi^5 W)) sum_{n odd} tanh(n pi W / (2H)) / n^5]."""
    s = sum(tanh(n * pi * W / (2 * H)) / n ** 5 for n in range(1, 2 * terms, 2))
    return g * H * H / (12 * nu) * (1 - 192 * H / (pi ** 5 * W) * s)


def test_duct_flow_rate_converges_to_continuum_poiseuille():
    """No-slip walls (r = 1 with the magic combination of the 2-D analysis):
    the mean velocity of a square duct approaches the continuum series
    solution at second order in the lattice spacing."""
    errs = []
    for n in (6, 12):
        kn = 0.1 * 12 / n         # the same viscosity in lattice units
        prm = D.Params3D(nx=1, ny=n, nz=n, kn=kn, gx=1e-6, r=1.0, A2=0.0, tq_den=24.0)
        P = _steady(prm, check=200, tol=1e-10)
        _, u = D.moments(P, prm)
        nu = C.tau_tilde(kn, n, 2.0) / 3.0
        errs.append(u[0].mean() / _duct_mean_velocity(n, n, 1e-6, nu) - 1)
    assert abs(errs[1]) < 0.008
    assert abs(errs[1]) < abs(errs[0]) / 3.5


def test_perturbed_window_is_part_of_the_start():
    prm = D.Params3D(nx=5, ny=7, nz=6)
    whole = D.init_perturbed(prm, 321, 1e-3)
    for y0, y1, z0, z1 in ((0, 3, 0, 3), (2, 7, 1, 4), (4, 5, 5, 6)):
        assert np.array_equal(D.init_perturbed_window(prm, 321, 1e-3, y0, y1, z0, z1), whole[:, z0:z1, y0:y1])


def _close(a, b):
    # the reference's back-transform solves a batch of linear systems, whose
    # last bits depend on the batch: agreement to rounding, not bit for bit
    return np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


@pytest.mark.parametrize("zbc", ["walls", "periodic"])
def test_windows_reproduce_the_duct(zbc):
    """Windows of full-width rows stepped on their own (rates from the duct's
    height) equal the whole duct's run on every row and layer more than n
    steps from a cut face: corner, edge and interior windows; a row next to a
    cut face does not."""
    nx, ny, nz, n = 6, 9, 8, 2
    prm = D.Params3D(nx=nx, ny=ny, nz=nz, zbc=zbc, kn=0.4, gx=1e-4, gy=2e-5, gz=-1e-5)
    P0 = D.init_perturbed(prm, 55, 1e-3)
    whole = D.run(P0, prm, n)
    w = 2 * n + 1
    # corner at y = 0, z = 0 (both walls in a duct): rows and layers 0 .. n
    got = D.run_window(P0[:, :w, :w].copy(), prm, n)
    if zbc == "walls":
        assert _close(got[:, :n + 1, :n + 1], whole[:, :n + 1, :n + 1])
    # top edge y = ny - 1 at interior layer zc: rows ny - n - 1 .. ny - 1 of layer zc
    zc = 4
    got = D.run_window(P0[:, zc - n:zc + n + 1, ny - w:].copy(), prm, n)
    assert _close(got[:, n, n:], whole[:, zc, ny - n - 1:])
    assert not _close(got[:, n, 0], whole[:, zc, ny - w])
    # interior: the middle row of the middle layer
    yc = 4
    got = D.run_window(P0[:, zc - n:zc + n + 1, yc - n:yc + n + 1].copy(), prm, n)
    assert _close(got[:, n, n], whole[:, zc, yc])
    assert not _close(got[:, 0, n], whole[:, zc - n, yc])
    # all layers of a z-periodic channel: z stays periodic, rows 0 .. n valid
    if zbc == "periodic":
        got = D.run_window(P0[:, :, :w].copy(), prm, n)
        assert _close(got[:, :, :n + 1], whole[:, :, :n + 1])


# ---------------------------------------------------------------------------
# Pressure-driven ducts (the 2-D inlet/outlet reading carried to 3-D).
# ---------------------------------------------------------------------------
def _pduct(**kw):
    base = dict(nx=9, ny=5, nz=4, xbc="pressure", kn=0.2, p_ratio=1.8)
    base.update(kw)
    return D.Params3D(**base)


def _opp_y(P):
    """Mirror y -> ny - 1 - y of populations (27, nz, ny, nx), directions b -> -b."""
    idx = [D.direction(a, -b, c) for a, b, c in D.E3]
    return P[idx][:, :, ::-1]


def _opp_z(P):
    idx = [D.direction(a, b, -c) for a, b, c in D.E3]
    return P[idx][:, ::-1]


def test_pressure_rest_state_is_steady():
    """Equal inlet and outlet pressure: the rest state is a fixed point."""
    prm = _pduct(p_ratio=1.0)
    P0 = D.init_linear_rho(prm)
    P = D.run(P0, prm, 5)
    assert np.max(np.abs(P - P0)) <= 1e-15


def test_pressure_linear_start_pull():
    """From the linear-density rest start the pull gives, at every column
    including the two next to the ghost planes, the node's own density and
    the momentum -(1/3) d rho/dx of the profile (interior rows and layers;
    the ghost density extrapolation makes the profile linear through the
    planes)."""
    prm = _pduct(nx=7, ny=5, nz=5, p_ratio=1.6)
    P = D.init_linear_rho(prm)
    pre = D.stream_bc(P, prm)
    rho, j = pre.sum(axis=0), np.tensordot(D.E3.T.astype(float), pre, (1, 0))
    x = np.arange(prm.nx) + 0.5
    rho_x = D.rho_in(prm) - (D.rho_in(prm) - prm.rho_out) * x / prm.nx
    inner = (slice(1, -1), slice(1, -1))
    assert np.max(np.abs(rho[inner] - rho_x)) <= 1e-14
    jx = (D.rho_in(prm) - prm.rho_out) / (3.0 * prm.nx)
    assert np.max(np.abs(j[0][inner] - jx)) <= 1e-14
    assert np.max(np.abs(j[1][inner])) <= 1e-14 and np.max(np.abs(j[2][inner])) <= 1e-14


def test_pressure_ghost_plane_moments():
    """Each ghost population row carries density 2 rho_b - rho_1 and
    velocity 2 u_1 - u_2 (moments computed from the populations), and its
    departure from its own equilibrium is that of the column next to it."""
    from clb_inputs import uniform_populations_3d
    prm = _pduct(nx=6, ny=4, nz=3, p_ratio=1.7, rho_out=1.1)
    P = uniform_populations_3d(6, 4, 3, seed=19) * 1.2
    g_in, g_out = D.ghost_planes(P, prm)
    for g, c1, c2, rb in ((g_in, 0, 1, D.rho_in(prm)), (g_out, 5, 4, prm.rho_out)):
        rho1, u1 = D.macroscopic(P[..., c1])
        _, u2 = D.macroscopic(P[..., c2])
        rg, ug = D.macroscopic(g)
        assert np.max(np.abs(rg - (2.0 * rb - rho1))) <= 1e-13
        assert np.max(np.abs(ug - (2.0 * u1 - u2))) <= 1e-12
        n = rho1.size
        eq_g = D.equilibrium(rg.ravel(), ug.reshape(3, n)).reshape(g.shape)
        eq_1 = D.equilibrium(rho1.ravel(), u1.reshape(3, n)).reshape(g.shape)
        assert np.max(np.abs((g - eq_g) - (P[..., c1] - eq_1))) <= 1e-13


def test_pressure_interior_equals_periodic_step_at_local_kn():
    """A state uniform along x: away from the ghost planes the pressure step
    equals the periodic duct's step at Kn = Kn_out rho_out / rho_c, rho_c the
    pre-collision density at the central nodes of the cross-section (odd and
    even heights and widths)."""
    from clb_inputs import uniform_populations_3d
    for ny, nz in ((5, 4), (4, 5), (6, 6), (3, 3)):
        prm = _pduct(nx=6, ny=ny, nz=nz, kn=0.3, p_ratio=1.5, rho_out=0.9)
        col = uniform_populations_3d(1, ny, nz, seed=3 + ny)        # (27, nz, ny, 1)
        P = np.repeat(col, prm.nx, axis=3)
        got = D.step(P, prm)
        per = D.Params3D(nx=prm.nx, ny=ny, nz=nz, kn=prm.kn)
        rho, _ = D.macroscopic(D.stream_bc(P, per))
        mid = {3: [1], 4: [1, 2], 5: [2], 6: [2, 3]}      # middle row(s) of 3 .. 6
        rho_c = rho[mid[nz]][:, mid[ny], 0].mean()
        per = dataclasses.replace(per, kn=prm.kn * prm.rho_out / rho_c)
        ref = D.step(P, per)
        assert np.max(np.abs(got[..., 1:-1] - ref[..., 1:-1])) <= 1e-14 * np.max(np.abs(ref)), (ny, nz)


def test_pressure_symmetry_and_z_uniformity():
    """The linear start of a duct stays mirror-symmetric in y and in z; that
    of a z-periodic channel stays uniform along z."""
    prm = _pduct(nx=8, ny=5, nz=4, p_ratio=1.9)
    P = D.run(D.init_linear_rho(prm), prm, 4)
    assert np.max(np.abs(P - _opp_y(P))) <= 1e-14
    assert np.max(np.abs(P - _opp_z(P))) <= 1e-14
    ch = _pduct(nx=8, ny=5, nz=3, zbc="periodic", p_ratio=1.9)
    P = D.run(D.init_linear_rho(ch), ch, 4)
    assert np.max(np.abs(P - P[:, :1])) <= 1e-15


def test_pressure_duct_reaches_uniform_mass_flow():
    """A short duct run from the linear start: the mass flow through every
    cross-section becomes the same (steady state), positive, from the inlet
    to the outlet."""
    prm = _pduct(nx=20, ny=4, nz=4, kn=0.1, p_ratio=1.5)
    P = D.run(D.init_linear_rho(prm), prm, 400)
    m = D.mass_flow(P, prm)
    assert m.min() > 0
    assert (m.max() - m.min()) / m.mean() <= 1e-6
