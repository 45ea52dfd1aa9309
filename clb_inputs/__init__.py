"""Seeded synthetic inputs and workload shapes for the CLB tests and benchmark.

Holds no arithmetic of the method itself: only array shapes, parameter sets
(the paper's values and the benchmark workloads) and seeded random numbers.
Both the HIP path and the CPU reference receive their inputs from here.
"""
import numpy as np

# Parameter values fixed in Section 3 of the paper (Liu & He, arXiv:1603.01955).
PAPER_A = 2.0
PAPER_B2 = 0.55
PAPER_S3 = 1.1
PAPER_S8 = 1.2


def uniform_populations(nx, ny, seed, lo=0.05, hi=0.15):
    """Random positive populations, shape (9, ny, nx), uniform in [lo, hi).

    Far from equilibrium on purpose: every moment of the collision is excited.
    """
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(9, ny, nx))


def uniform_populations_3d(nx, ny, nz, seed, lo=0.02, hi=0.06):
    """Random positive D3Q27 populations, shape (27, nz, ny, nx), uniform in
    [lo, hi) (density about 1, far from equilibrium)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(27, nz, ny, nx))


def sample_nodes(nx, ny, count, seed):
    """Distinct node coordinates (ys, xs): all four corners, the wall rows,
    the first and last columns, plus uniform random interior picks."""
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1),
             (0, nx // 2), (ny - 1, nx // 2), (ny // 2, 0), (ny // 2, nx - 1)]
    ys = rng.integers(0, ny, size=count)
    xs = rng.integers(0, nx, size=count)
    pts = sorted(set(fixed) | set(zip(ys.tolist(), xs.tolist())))
    return (np.array([p[0] for p in pts], dtype=np.int64),
            np.array([p[1] for p in pts], dtype=np.int64))


def kn_sweep_channels(count=64, seed=7, heights=(16, 24, 32, 48, 64, 96, 128),
                      kn_lo=0.01, kn_hi=10.0):
    """Batched Kn-sweep workload: ``count`` periodic channels with Kn
    log-spaced over [kn_lo, kn_hi] and heights drawn from ``heights``."""
    rng = np.random.default_rng(seed)
    ny = rng.choice(np.array(heights), size=count)
    kn = kn_lo * (kn_hi / kn_lo) ** (np.arange(count) / max(count - 1, 1))
    return [int(v) for v in ny], [float(v) for v in kn]


def kn_minimum_channels(count=48, ny=32, kn_lo=0.3, kn_hi=3.0):
    """A single-height Kn sweep around the Knudsen minimum: ``count``
    periodic channels of ``ny`` rows with Kn log-spaced over [kn_lo, kn_hi]
    (Q depends on the height too, so its minimum over Kn is read off
    channels of one height)."""
    kn = kn_lo * (kn_hi / kn_lo) ** (np.arange(count) / max(count - 1, 1))
    return [int(ny)] * count, [float(v) for v in kn]


# Pressure ratio and TMAC of the paper's mass-flow study (Section 3.2).
MASS_FLOW_P_RATIO = 1.8
MASS_FLOW_SIGMA = 0.93


def mass_flow_sweep_kn(count=16, kn_lo=0.01, kn_hi=1.0):
    """Outlet Knudsen numbers of the pressure-driven mass-flow sweep:
    ``count`` values log-spaced over [kn_lo, kn_hi] (the study covers Kn_out
    up to about 0.5 and Kn_ave up to about 0.8)."""
    kn = kn_lo * (kn_hi / kn_lo) ** (np.arange(count) / max(count - 1, 1))
    return [float(v) for v in kn]


# Workloads (sizes follow the paper's two test problems, Section 3).
WORKLOADS = {
    # Force-driven periodic channel, small: steady state after 20,000 steps.
    "channel_4x32": dict(nx=4, ny=32, xbc="periodic", kn=0.1, gx=1e-6, steps=20000),
    # Long pressure-driven channel, L/H = 100.
    "long_4000x40": dict(nx=4000, ny=40, xbc="pressure", kn=0.1, p_ratio=2.0, steps=200000),
    # Large periodic channel used for throughput.
    "periodic_32768x2048": dict(nx=32768, ny=2048, xbc="periodic", kn=1.0, gx=1e-7,
                                init="perturbed", init_amp=1e-4, seed=12345),
    # Long channel for the adjoint calibration, L/H = 100.
    "long_2000x20": dict(nx=2000, ny=20, xbc="pressure", kn=0.1, p_ratio=2.0, steps=2000),
    # Rectangular microduct (3-D extension): square cross-section, force driven.
    "duct_512x256x256": dict(nx=512, ny=256, nz=256, kn=0.5, gx=1e-6, init="perturbed", init_amp=1e-4,
                             seed=2468),
    # Long pressure-driven microduct (3-D extension of the long channel): square
    # 40 x 40 cross-section, L/H = 100, p_in/p_out = 2, Kn_out = 0.1.
    "duct_pressure_4000x40x40": dict(nx=4000, ny=40, nz=40, xbc="pressure", kn=0.1, p_ratio=2.0,
                                     init="linear_rho"),
    # Mass-flow sweep: 16 long channels, L/H = 100, Kn_out 0.01 .. 1.
    "mass_flow_sweep_16x2000x20": dict(nx=2000, ny=20, xbc="pressure", p_ratio=MASS_FLOW_P_RATIO,
                                       sigma=MASS_FLOW_SIGMA, channels=16, kn_lo=0.01, kn_hi=1.0),
}
