"""GPU tests of the batch of pressure-driven channels (the mass-flow study of
Section 3.2 of Liu & He, arXiv:1603.01955), through the C ABI.

Each channel must match the CPU reference element by element over its first
steps (every launch shape the batch can take), advance bitwise as a
single-channel context with the same parameters, stop at the first check
where its mass flow has settled, and the converged sweep's dimensionless
mass flow S = m / m_ns must follow the lubrication model of the scheme.  The
paper prints no numbers for this study (its figure compares with external
data), so agreement with the paper itself is unpinned.
"""
import numpy as np
import pytest
import torch

from clb_inputs import MASS_FLOW_P_RATIO, MASS_FLOW_SIGMA, mass_flow_sweep_kn
from oracle import analytic as A
from oracle import clb_ref as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")


def _mods():
    from paper_1603_01955_amd import PressureBatch, Solver, clb
    return PressureBatch, Solver, clb


# Per-channel parameter variety: slip coefficients, rates, pressures, start.
MIXED = [
    dict(kn=0.05, p_ratio=1.8, sigma=0.93),
    dict(kn=0.2, p_ratio=2.0, A2=0.3, tq_den=24.0),
    dict(kn=0.8, p_ratio=1.5, sigma=0.8, rho_out=1.3),
    dict(kn=0.1, p_ratio=2.5, r=0.9, a=1.0, s3=1.3, s8=0.9, init="uniform"),
]


def _specs(nch):
    out = []
    for c in range(nch):
        d = dict(MIXED[c % len(MIXED)])
        d["kn"] *= 1.0 + 0.1 * c
        out.append(d)
    return out


def _gpu_params(clb, nx, ny, spec, shift=1):
    return clb.make_params(nx, ny, xbc="pressure", cbbsr_shift=shift, **spec)


def _ref(nx, ny, spec, shift=1):
    d = dict(spec)
    init = d.pop("init", "linear_rho")
    prm = C.Params(nx=nx, ny=ny, xbc="pressure", cbbsr_shift=shift, **d)
    P0 = C.init_uniform(prm) if init == "uniform" else C.init_linear_rho(prm)
    return prm, P0


@pytest.mark.parametrize("nx,ny,nch,steps,shift,path", [
    (149, 12, 4, 30, 1, 1),    # column kernel: 256-thread workgroups, 16 row lanes
    (1030, 40, 5, 8, 1, 1),    # 1024-thread workgroups, 64 row lanes
    (500, 20, 8, 6, 1, 1),     # 512-thread workgroups, 32 row lanes
    (50, 70, 2, 10, 0, 1),     # ny > 64: several rows per thread; literal Eq. (20) source
    (2, 3, 3, 5, 1, 1),        # one workgroup per channel holds both ghost columns
    (149, 12, 4, 30, 1, 2),    # row kernel (prep + row streaming)
    (1030, 40, 3, 8, 0, 2),    # row kernel, two row segments per row
])
def test_matches_reference(nx, ny, nch, steps, shift, path):
    PressureBatch, _, clb = _mods()
    specs = _specs(nch)
    pb = PressureBatch([_gpu_params(clb, nx, ny, s, shift) for s in specs])
    pb.set_path(path)
    pb.step(steps)
    m, m_ns = pb.massflow()
    for c, spec in enumerate(specs):
        prm, P0 = _ref(nx, ny, spec, shift)
        Pref = C.run(P0, prm, steps)
        P = pb.populations(c).cpu().numpy()
        assert np.max(np.abs(P - Pref)) <= 1e-10 * np.max(np.abs(Pref)), c
        mref, suref, rcref = C.column_sums(Pref, prm)
        mx, su, rc = (t.cpu().numpy() for t in pb.column_sums(c))
        scale = np.max(np.abs(mref))
        assert np.max(np.abs(mx - mref)) <= 1e-10 * scale, c
        assert np.max(np.abs(rc - rcref)) <= 1e-12, c
        assert abs(m[c] - mref.mean()) <= 1e-10 * scale, c
        dp = pb.pressure_deviation(c).cpu().numpy()
        assert np.max(np.abs(dp - C.pressure_deviation(Pref, prm))) <= 1e-10, c
        want_ns = A.noslip_massflow(nx, ny, prm.kn, prm.p_ratio, rho_out=prm.rho_out)
        assert abs(m_ns[c] / want_ns - 1.0) <= 1e-14, c
    pb.close()


def test_bench_workload_matches_reference():
    """The benchmarked mass-flow sweep itself (16 channels 2000 x 20, ratio
    1.8, sigma 0.93, Kn_out 0.01-1, the launch shape bench.py times): every
    channel against the CPU reference after 4 steps, element by element."""
    PressureBatch, _, clb = _mods()
    nx, ny = 2000, 20
    kns = mass_flow_sweep_kn(16)
    specs = [dict(kn=k, p_ratio=MASS_FLOW_P_RATIO, sigma=MASS_FLOW_SIGMA) for k in kns]
    pb = PressureBatch([_gpu_params(clb, nx, ny, s) for s in specs])
    pb.step(4)
    for c, spec in enumerate(specs):
        prm, P0 = _ref(nx, ny, spec)
        Pref = C.run(P0, prm, 4)
        P = pb.populations(c).cpu().numpy()
        assert np.max(np.abs(P - Pref)) <= 1e-10 * np.max(np.abs(Pref)), c
    pb.close()


@pytest.mark.parametrize("nx,ny,nch", [(149, 12, 4), (1030, 40, 5), (50, 70, 2), (2, 3, 3), (2000, 20, 3)])
def test_row_and_column_kernels_agree_bitwise(nx, ny, nch):
    """Row and column kernels, one to four steps per launch (odd chunks, so
    every launch kind, shorter remainders and both buffers occur): the same
    populations."""
    PressureBatch, _, clb = _mods()
    params = [_gpu_params(clb, nx, ny, s) for s in _specs(nch)]
    out = []
    for path in (1, 2):
        for spl in ((1, 2, 3, 4) if path == 1 else (1, 2)):
            pb = PressureBatch(params)
            pb.set_path(path)
            pb.set_steps_per_launch(spl)
            pb.step(7)
            steps, _ = pb.run(6, check_every=3, tol=0.0)
            assert steps.tolist() == [13] * nch
            out.append([pb.populations(c) for c in range(nch)])
            pb.close()
    for k in range(1, len(out)):
        for c in range(nch):
            assert torch.equal(out[0][c], out[k][c]), (k, c)


def test_run_stops_each_channel_where_its_mass_flow_settles():
    """Checks every 500 steps with tol = 1e-5: each channel stops at the first
    check whose mass flow is within tol of the previous one, and its state
    equals a single-channel solver's after that many steps, bit for bit."""
    PressureBatch, Solver, clb = _mods()
    nx, ny, every, tol = 300, 10, 500, 1e-5
    specs = [dict(kn=k, p_ratio=1.8, sigma=0.93) for k in (0.02, 0.1, 0.5, 2.0)]
    params = [_gpu_params(clb, nx, ny, s) for s in specs]
    pb = PressureBatch(params)
    steps, conv = pb.run(200000, check_every=every, tol=tol)
    assert conv.all(), steps
    assert len(set(steps.tolist())) > 1, steps        # the channels stop at different checks
    assert np.all(steps % every == 0)
    m, _ = pb.massflow()
    for c in range(len(params)):
        s = Solver(params=params[c])
        s.set_graph_steps(every)
        hist = []
        for _ in range(steps[c] // every):
            s.step(every)
            hist.append(s.massflow()[1])
        assert torch.equal(s.populations(), pb.populations(c)), c
        assert abs(m[c] - hist[-1]) <= 1e-13 * abs(hist[-1]), c
        assert abs(hist[-1] - hist[-2]) <= tol * abs(hist[-1]), c
        if len(hist) >= 3:
            assert abs(hist[-2] - hist[-3]) > tol * abs(hist[-2]), c
        s.close()
    pb.close()


def test_step_and_odd_chunks_keep_buffers_straight():
    """Plain steps, then a run whose odd chunk length replays the graphs of
    both starting buffers plus a shorter tail: every channel equals a
    single-channel solver after the same number of steps."""
    PressureBatch, Solver, clb = _mods()
    nx, ny = 64, 6
    params = [_gpu_params(clb, nx, ny, s) for s in _specs(3)]
    pb = PressureBatch(params)
    pb.step(3)
    steps, conv = pb.run(10, check_every=3, tol=0.0)
    assert steps.tolist() == [13, 13, 13] and not conv.any()
    steps, _ = pb.run(5)
    assert steps.tolist() == [18, 18, 18]
    steps, _ = pb.run(9, check_every=3, tol=0.0)     # same graphs, replayed
    assert steps.tolist() == [27, 27, 27]
    for c, p in enumerate(params):
        s = Solver(params=p)
        s.step(27)
        assert torch.equal(s.populations(), pb.populations(c)), c
        s.close()
    pb.close()


def test_set_populations_and_failure_detection():
    """A channel given the reference's state continues like the reference; a
    channel given a non-finite value is reported by check_finite and stays
    confined to itself (channels are independent)."""
    PressureBatch, _, clb = _mods()
    nx, ny = 60, 8
    specs = _specs(3)
    pb = PressureBatch([_gpu_params(clb, nx, ny, s) for s in specs])
    pb.step(3)
    assert pb.check_finite().all()
    prm, P0 = _ref(nx, ny, specs[0])
    Pmid = C.run(P0, prm, 5)
    pb.set_populations(0, torch.from_numpy(Pmid))
    bad = pb.populations(1).clone()
    bad[4, 3, 7] = float("nan")
    pb.set_populations(1, bad)
    assert pb.check_finite().tolist() == [True, False, True]
    pb.step(4)
    assert pb.check_finite().tolist() == [True, False, True]
    P = pb.populations(0).cpu().numpy()
    Pref = C.run(Pmid, prm, 4)
    assert np.max(np.abs(P - Pref)) <= 1e-10 * np.max(np.abs(Pref))
    pb.close()


def test_zero_steps_and_converged_channels_do_not_move():
    PressureBatch, _, clb = _mods()
    params = [_gpu_params(clb, 40, 4, s) for s in _specs(2)]
    pb = PressureBatch(params)
    P0 = [pb.populations(c).clone() for c in range(2)]
    pb.step(0)
    steps, conv = pb.run(0, check_every=10, tol=1.0)
    assert steps.tolist() == [0, 0] and not conv.any()
    for c in range(2):
        assert torch.equal(pb.populations(c), P0[c])
    # tol = 1: every channel stops at an early check and stays there
    steps1, conv = pb.run(200, check_every=10, tol=1.0)
    assert conv.all() and np.all(steps1 % 10 == 0) and np.all(steps1 >= 20), steps1
    P1 = [pb.populations(c).clone() for c in range(2)]
    pb.step(7)
    steps2, conv = pb.run(50, check_every=10, tol=1.0)
    assert steps2.tolist() == steps1.tolist()
    for c in range(2):
        assert torch.equal(pb.populations(c), P1[c])
    pb.close()


@pytest.fixture(scope="module")
def sweep():
    """The mass-flow study at L/H = 100 (2000 x 20), pressure ratio 1.8,
    sigma = 0.93, six outlet Knudsen numbers, run to steady state."""
    PressureBatch, _, clb = _mods()
    nx, ny = 2000, 20
    kns = mass_flow_sweep_kn(count=6, kn_lo=0.02, kn_hi=1.0)
    pb = PressureBatch([_gpu_params(clb, nx, ny, dict(kn=k, p_ratio=MASS_FLOW_P_RATIO, sigma=MASS_FLOW_SIGMA))
                        for k in kns])
    steps, conv = pb.run(3000000, check_every=2000, tol=1e-10)
    yield nx, ny, kns, pb, steps, conv
    pb.close()


def test_sweep_reaches_uniform_mass_flow(sweep):
    """Every channel settles; its column mass flow is uniform along the
    channel up to the steady discrete structure near the inlet and outlet,
    which grows with the relaxation time (below 1e-5 of the mean here)."""
    nx, ny, kns, pb, steps, conv = sweep
    assert conv.all(), steps
    spread = []
    for c in range(len(kns)):
        mx = pb.column_sums(c)[0].cpu().numpy()
        spread.append((mx.max() - mx.min()) / mx.mean())
    assert max(spread) <= 2e-5, (spread, steps)
    assert np.all(np.diff(spread) > 0), spread


def test_sweep_dimensionless_mass_flow_follows_lubrication_model(sweep):
    """S = m / m_ns grows with Kn_out and follows the lubrication model with
    the slip law of Eq. (19) and the Bosanquet viscosity (second-order slip
    coefficient 12 B2) within 0.3% from Kn_out = 0.05, within 1.5% below
    (where the flow is fastest and the model's neglect of inertia shows).
    The force-driven channel's discrete slip excess (18 B2) is absent: that
    model is more than 5% off at Kn_out = 1."""
    nx, ny, kns, pb, steps, conv = sweep
    m, m_ns = pb.massflow()
    S = m / m_ns
    assert np.all(np.diff(S) > 0), S
    A1 = C.slip_A1(MASS_FLOW_SIGMA)

    def s_lub(k, c2):
        m_lub, _ = A.lubrication_profile(nx, ny, k, MASS_FLOW_P_RATIO, 2.0, A1, 0.55, nsub=1, c2=c2)
        return m_lub / A.noslip_massflow(nx, ny, k, MASS_FLOW_P_RATIO)

    for c, k in enumerate(kns):
        tol = 0.003 if k >= 0.05 else 0.015
        assert abs(S[c] / s_lub(k, 12.0) - 1.0) <= tol, (k, S[c], s_lub(k, 12.0))
    assert S[-1] / s_lub(kns[-1], 18.0) < 0.95
