"""GPU tests of the batched Kn-sweep form, through the C ABI.

Each channel of a batch must advance bitwise identically to a single-channel
context with the same parameters (same gather and collision code), match the
CPU reference, and the converged sweep must reproduce the closed-form
steady flow rate of the scheme and its Knudsen minimum (Section 3.1).
"""
import numpy as np
import pytest
import torch

from clb_inputs import kn_minimum_channels, kn_sweep_channels, uniform_populations
from oracle import analytic as A
from oracle import clb_ref as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")


def _mods():
    from paper_1603_01955_amd import Batch, Solver, clb
    return Batch, Solver, clb


CHANNELS = [
    dict(nx=4, ny=16, kn=0.3, gx=1e-6),
    dict(nx=6, ny=24, kn=0.05, gx=1e-6, forcing=1),     # third-order force moments; 144 nodes > 64 threads
    dict(nx=4, ny=128, kn=0.01, gx=1e-6),
    dict(nx=7, ny=9, kn=2.0, gx=1e-4, gy=3e-5, cbbsr_shift=0),
    dict(nx=1, ny=1, kn=0.5, gx=1e-5),
    dict(nx=32, ny=32, kn=10.0, gx=1e-6, sigma=0.8, tq_den=24.0),
    dict(nx=3, ny=5, kn=0.1, init="perturbed", init_amp=1e-3, seed=9),
    dict(nx=5, ny=12, kn=0.7, gx=2e-5, gy=1e-5, forcing=1),          # third-order force moments
]


def test_batch_bitwise_equals_single_channel():
    Batch, Solver, clb = _mods()
    params = [clb.make_params(**kw) for kw in CHANNELS]
    b = Batch(params)
    starts = {}
    for c, kw in enumerate(CHANNELS):
        if c % 2 == 0:   # random far-from-equilibrium start on half the channels
            starts[c] = uniform_populations(kw["nx"], kw["ny"], seed=200 + c)
            b.set_populations(c, torch.from_numpy(starts[c]))
    steps, conv = b.run(137)
    assert (steps == 137).all() and not conv.any()
    for c, kw in enumerate(CHANNELS):
        s = Solver(params=clb.make_params(**kw))
        if c in starts:
            s.set_populations(torch.from_numpy(starts[c]))
        s.step(137)
        assert torch.equal(b.populations(c), s.populations()), c


def test_batch_matches_reference():
    Batch, _, clb = _mods()
    b = Batch([clb.make_params(**kw) for kw in CHANNELS])
    b.run(60)
    for c, kw in enumerate(CHANNELS):
        keys = {k: v for k, v in kw.items() if k not in ("init", "init_amp", "seed")}
        prm = C.Params(**keys)
        P0 = C.init_perturbed(prm, 9, 1e-3) if kw.get("init") == "perturbed" else C.init_uniform(prm)
        ref = C.run(P0, prm, 60)
        got = b.populations(c).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref)), c


def test_graph_replay_continues_and_tuner_leaves_state():
    Batch, _, clb = _mods()
    params = [clb.make_params(**kw) for kw in CHANNELS[:4]]
    one = Batch(params)
    one.run(200)
    two = Batch(params)
    t, o = two.tune(probe_steps=50)
    assert t in (64, 128, 256, 512, 1024) and o in (0, 1)
    steps, _ = two.run(100)
    assert (steps == 100).all()
    steps, _ = two.run(100)          # replay of the recorded graph
    assert (steps == 200).all()
    for c in range(len(params)):
        assert torch.equal(one.populations(c), two.populations(c))
    for threads in (64, 1024):
        for longest in (0, 1):
            three = Batch(params)
            three.set_launch(threads, longest)
            three.run(200)
            for c in range(len(params)):
                assert torch.equal(one.populations(c), three.populations(c)), (threads, longest)


def test_kn_sweep_matches_closed_form_and_knudsen_minimum():
    """64 periodic channels, heights from {16..128}, Kn log-spaced 0.01-10,
    g = 1e-6, each run to steady state in one persistent launch."""
    Batch, _, clb = _mods()
    heights, kns = kn_sweep_channels(64, seed=7)
    params = [clb.make_params(4, ny, kn=kn, gx=1e-6) for ny, kn in zip(heights, kns)]
    b = Batch(params)
    b.tune(probe_steps=200)
    steps, conv = b.run(400000, check_every=1000, tol=1e-12)
    assert conv.all(), steps[~conv]
    Q = b.flow_rate()
    r = C.bounce_fraction(C.slip_A1(1.0))
    Qref = np.array([A.discrete_Q(ny, kn, 2.0, 0.55, r) for ny, kn in zip(heights, kns)])
    assert np.max(np.abs(Q / Qref - 1)) <= 1e-6


def test_knudsen_minimum_from_gpu_flow_rates():
    """The Knudsen minimum read off the GPU's own steady flow rates: 48
    channels of one height (ny = 32), Kn log-spaced over [0.3, 3] (a 5% grid),
    one persistent launch.  The GPU's Q falls, then rises, with its smallest
    value within one grid cell of the scheme's closed-form minimum (0.87 for
    this height), which brackets the paper's Kn ~ 0.9 (Section 3.1)."""
    Batch, _, clb = _mods()
    heights, kns = kn_minimum_channels(48, ny=32, kn_lo=0.3, kn_hi=3.0)
    b = Batch([clb.make_params(4, ny, kn=kn, gx=1e-6) for ny, kn in zip(heights, kns)])
    steps, conv = b.run(400000, check_every=1000, tol=1e-12)
    assert conv.all(), steps[~conv]
    Q = b.flow_rate()
    grid = np.array(kns)
    k = int(np.argmin(Q))
    assert 0 < k < len(grid) - 1
    assert np.all(np.diff(Q[:k + 1]) < 0) and np.all(np.diff(Q[k:]) > 0)
    r = C.bounce_fraction(C.slip_A1(1.0))
    fine = np.exp(np.linspace(np.log(0.3), np.log(3.0), 4001))
    kstar = fine[int(np.argmin([A.discrete_Q(32, kn, 2.0, 0.55, r) for kn in fine]))]
    cell = grid[1] / grid[0]
    assert kstar / cell <= grid[k] <= kstar * cell
    assert 0.8 < grid[k] < 0.95


def test_kn_sweep_with_third_order_forcing_matches_continuum_slip():
    """The same sweep shape with the source's third-order moments: every
    channel's steady Q is the continuum second-order slip solution of
    Eq. (19) (discrete excess of Eq. (9)'s source removed)."""
    Batch, _, clb = _mods()
    heights, kns = kn_sweep_channels(16, seed=11, heights=(16, 32, 64))
    params = [clb.make_params(4, ny, kn=kn, gx=1e-6, forcing=1) for ny, kn in zip(heights, kns)]
    b = Batch(params)
    steps, conv = b.run(400000, check_every=1000, tol=1e-12)
    assert conv.all(), steps[~conv]
    Q = b.flow_rate()
    A1 = C.slip_A1(1.0)
    Qref = np.array([A.continuum_sum_u(ny, kn, 2.0, A1, 0.55, 1e-6) * np.sqrt(6.0) / (3.0 * 1e-6 * ny * ny)
                     for ny, kn in zip(heights, kns)])
    assert np.max(np.abs(Q / Qref - 1)) <= 1e-6


def test_batch_failure_detection():
    """A planted non-finite value is reported for its channel only, also
    after further steps (channels are independent)."""
    Batch, _, clb = _mods()
    params = [clb.make_params(**kw) for kw in CHANNELS[:3]]
    b = Batch(params)
    b.run(10)
    assert b.check_finite().all()
    bad = b.populations(1).clone()
    bad[2, 5, 3] = float("inf")
    b.set_populations(1, bad)
    assert b.check_finite().tolist() == [True, False, True]
    b.run(10)
    assert b.check_finite().tolist() == [True, False, True]
    b.close()


def test_batch_rejects_bad_channels():
    Batch, _, clb = _mods()
    with pytest.raises(clb.ClbError):
        Batch([clb.make_params(10, 8, xbc="pressure")])
    with pytest.raises(clb.ClbError):
        Batch([clb.make_params(512, 512, kn=1.0, gx=1e-6)])   # does not fit in LDS
