"""Benchmark of the fused D2Q9 cascaded LB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: periodic force-driven channel, 32768 x 2048 nodes (H = 2048),
Kn = 1, body acceleration 1e-7, seeded perturbed equilibrium start, FP64.
A step is one full pass of the hot path over the grid: pull streaming with
periodic x and CBBSR slip walls, cascaded collision with forcing.  Prints
one JSON line.
"""
import argparse
import json
import os
import sys
import time

METRIC = "D2Q9 CLB MLUPS & HBM GB/s; batched Kn-sweep vs loop; adjoint/forward time"
WORKLOAD = dict(nx=32768, ny=2048, kn=1.0, gx=1e-7, init="perturbed", init_amp=1e-4, seed=12345)
BYTES_PER_NODE = 144          # 9 FP64 loads + 9 FP64 stores per node update
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E, published
# FP64 vector issue: one wave64 FP64 instruction per clock per CU
# (78.6 TFLOP/s = 256 CUs x 2.4 GHz x 64 lanes x 2 flops per FMA).
FP64_WAVE_INSTS_PER_S = 256 * 2.4e9
CPU_SAMPLE_NX = 512           # full-height slab of the workload: wall rows 2 of 2048, as on the full grid
CPU_SAMPLE_STEPS = 15


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batched Kn-sweep comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--part", choices=("all", "step", "sweep", "pressure", "msweep", "adjoint", "duct", "pduct"),
                    default="all",
                    help="run one part alone (step: the periodic step only, at the chosen steps per launch alone; sweep / pressure / msweep / adjoint / "
                         "duct (force-driven 3-D duct) / pduct (pressure-driven 3-D duct): that measurement only, "
                         "printed as its own JSON line) -- for profiling runs")
    ap.add_argument("--no-loop-baseline", action="store_true",
                    help="sweep / msweep: skip the loop-of-solvers baselines (profiling the batched kernel)")
    ap.add_argument("--no-msweep", action="store_true", help="skip the pressure-driven mass-flow sweep")
    ap.add_argument("--msweep-max-steps", type=int, default=3000000,
                    help="msweep: step cap per channel (lower it for traced runs)")
    ap.add_argument("--steps-per-launch", type=int, default=3,
                    help="periodic step: steps per launch (1-4; the earlier ones kept in LDS)")
    ap.add_argument("--channel-steps-per-launch", type=int, default=None,
                    help="pressure and msweep parts: steps per launch (default: the library's)")
    ap.add_argument("--pressure-steps", type=int, default=200000,
                    help="pressure: steps of the long-channel run (2e5 is the paper's run; fewer for traced runs)")
    ap.add_argument("--block-x", type=int, default=1024)
    ap.add_argument("--xcd-remap", type=int, default=1)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="instead of the benchmark, run a plain device copy of this many GB "
                         "(reference kernel for scaling hardware byte counters)")
    return ap.parse_args()


def copy_calibration(gb):
    """A plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
    calibrate the counters read on the step kernel (the library's copy
    kernel, k_copy16, three launches)."""
    import torch
    from paper_1603_01955_amd.clb import hbm_copy
    n = int(gb * 1e9) // 16 * 2
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        hbm_copy(src, dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)


def profile_record():
    """Per-launch counter figures of the step kernel from the committed
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a
    plain copy of known size; FP64 VALU instructions), or {} unless they were
    taken on the current kernel sources."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "step_periodic_32768x2048_traffic.txt")
    rec = {}
    try:
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    rec[k.strip()] = v.strip()
    except OSError:
        return {}
    from paper_1603_01955_amd.build import source_hash
    if rec.get("source_hash") != source_hash():
        return {}
    return rec


def copy_bandwidth(gb=4.0, reps=10):
    """HBM ceiling measured on this GPU: the library's plain copy kernel
    (clb_hbm_copy, 16 bytes per thread) over gb GB, bytes read + written over
    the time of reps copies (HIP events on the stream it runs on)."""
    import torch
    from paper_1603_01955_amd.clb import hbm_copy
    n = int(gb * 1e9) // 16 * 2
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        hbm_copy(src, dst)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        hbm_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / s / 1e9


def kn_sweep(max_steps=400000, check_every=1000, tol=1e-12, baselines=True, forcing=0):
    """Batched Kn sweep (64 periodic channels, heights from {16..128}, Kn
    log-spaced 0.01-10, g = 1e-6, each to steady state) in one persistent
    launch, against a loop of single-channel solvers with the same check
    cadence, eager and hipGraph'd.  Returns a dict for the JSON line."""
    import numpy as np
    import torch
    from clb_inputs import kn_sweep_channels
    from paper_1603_01955_amd import Batch, Solver, clb

    heights, kns = kn_sweep_channels(64, seed=7)
    params = [clb.make_params(4, ny, kn=kn, gx=1e-6, forcing=forcing) for ny, kn in zip(heights, kns)]
    b = Batch(params)
    t0 = time.perf_counter()
    threads, longest = b.tune(probe_steps=200)
    t_tune = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_b, conv = b.run(max_steps, check_every, tol)        # synchronises
    t_batch = time.perf_counter() - t0
    q = b.flow_rate()
    b.close()

    def loop(graph):
        solvers = [Solver(params=p) for p in params]
        for s in solvers:
            if graph:
                s.set_graph_steps(check_every)
        torch.cuda.synchronize()
        steps = []
        t0 = time.perf_counter()
        for s in solvers:
            prev, n = float("nan"), 0
            while n < max_steps:
                s.step(check_every)
                n += check_every
                cur = s.flow_rate()                            # synchronises
                if abs(cur - prev) <= tol * abs(cur):
                    break
                prev = cur
            steps.append(n)
        dt = time.perf_counter() - t0
        for s in solvers:
            s.close()
        return dt, steps

    updates = int(sum(4 * int(ny) * int(n) for ny, n in zip(heights, steps_b)))   # node updates
    if not baselines:
        return {"channels": len(params), "all_converged": bool(conv.all()),
                "steps_total": int(steps_b.sum()), "node_updates": updates, "batched_s": round(t_batch, 4),
                "batched_mlups": round(updates / t_batch / 1e6, 1)}
    t_loop, steps_l = loop(graph=False)
    t_graph, _ = loop(graph=True)
    return {
        "channels": len(params), "check_every": check_every, "tol": tol,
        "all_converged": bool(conv.all()),
        "steps_total": int(steps_b.sum()), "steps_max": int(steps_b.max()), "node_updates": updates,
        "batched_mlups": round(updates / t_batch / 1e6, 1),
        "loop_steps_match": bool((np.array(steps_l) == steps_b).all()),
        "batched_s": round(t_batch, 4), "loop_s": round(t_loop, 4), "graph_loop_s": round(t_graph, 4),
        "speedup_vs_loop": round(t_loop / t_batch, 2), "speedup_vs_graph_loop": round(t_graph / t_batch, 2),
        "tuned": {"threads": threads, "longest_first": longest, "tune_s": round(t_tune, 3)},
        "cpu_oracle": kn_sweep_oracle(heights, kns, forcing),
    }


def kn_sweep_oracle(heights, kns, forcing):
    """The CPU reference on the sweep's tallest channel, the one that sets
    the batch's time (the reference steps channels one at a time)."""
    import numpy as np
    from oracle import clb_ref as C
    j = int(np.argmax(heights))
    prm = C.Params(nx=4, ny=int(heights[j]), kn=float(kns[j]), gx=1e-6, forcing=forcing)
    st = {"P": C.init_uniform(prm)}

    def step():
        st["P"] = C.step(st["P"], prm)
    return oracle_rate(step, prm.nx * prm.ny, "the 4 x %d channel at Kn = %.3g" % (prm.ny, prm.kn), budget_s=2.0)


def kn_minimum(ny=64, count=48, kn_lo=0.3, kn_hi=3.0, forcing=0, max_steps=400000, check_every=1000,
               tol=1e-12):
    """The Knudsen minimum of the flow rate (Section 3.1) read off one batched
    launch of channels of a single height (Q depends on the height too):
    count channels 4 x ny, Kn log-spaced over [kn_lo, kn_hi], g = 1e-6, each
    to steady state.  Reports the Kn of the smallest steady Q and the grid
    spacing."""
    import numpy as np
    from clb_inputs import kn_minimum_channels
    from paper_1603_01955_amd import Batch, clb

    heights, kns = kn_minimum_channels(count, ny=ny, kn_lo=kn_lo, kn_hi=kn_hi)
    b = Batch([clb.make_params(4, h, kn=k, gx=1e-6, forcing=forcing) for h, k in zip(heights, kns)])
    t0 = time.perf_counter()
    steps, conv = b.run(max_steps, check_every, tol)
    dt = time.perf_counter() - t0
    q = b.flow_rate()
    b.close()
    k = int(np.argmin(q))
    return {"ny": ny, "channels": count, "kn_range": [kn_lo, kn_hi], "grid_ratio": round(kns[1] / kns[0], 4),
            "all_converged": bool(conv.all()), "steps_max": int(steps.max()), "batched_s": round(dt, 4),
            "kn_at_min_Q": round(kns[k], 4), "Q_min": round(float(q[k]), 6),
            "interior_minimum": bool(0 < k < count - 1)}


def adjoint_calibration(T=2000, K=45, repeats=3):
    """Adjoint of the long pressure-driven channel (L/H = 100, 2000 x 20,
    p_in/p_out = 2, Kn_out = 0.1) over T steps with K-step checkpoints: the
    target (dp*, m*) comes from the same run with theta* = theta0 (1 + 0.05 xi),
    xi ~ N(0, 1) seeded 2024, over theta = (a, A1, A2, r).  Times the forward
    run (with checkpoints and loss) and the backward sweep (recompute + reverse)."""
    import numpy as np
    import torch
    from paper_1603_01955_amd import Adjoint, clb

    A1 = 1.0 - 0.1817          # sigma = 1 (Section 3)
    r0 = 1.0 / (1.0 + A1 * np.sqrt(np.pi / 6.0))
    theta0 = np.array([2.0, A1, 0.55, r0])
    xi = np.random.default_rng(2024).standard_normal(4)
    star = theta0 * (1.0 + 0.05 * xi)

    def params(th):
        return clb.make_params(2000, 20, xbc="pressure", kn=0.1, p_ratio=2.0,
                               a=th[0], A1=th[1], A2=th[2], r=th[3])

    tgt = Adjoint(params(star), T, K)
    tgt.forward(torch.zeros(2000, dtype=torch.float64), 1.0)
    dps, ms = tgt.observables()
    tgt.close()
    adj = Adjoint(params(theta0), T, K)
    adj.forward(dps, ms)          # warm-up (first launches, graph-free)
    adj.backward()
    tf, tb = [], []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = adj.forward(dps, ms)             # synchronises
        t1 = time.perf_counter()
        g = adj.backward()                      # synchronises
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tb.append(t2 - t1)
    adj.close()
    f, b = min(tf), min(tb)
    from threadpoolctl import threadpool_limits
    from oracle import adjoint_ref as AR
    from oracle import clb_ref as C
    prm = C.Params(nx=2000, ny=20, xbc="pressure", kn=0.1, p_ratio=2.0, a=theta0[0], A1=theta0[1], A2=theta0[2],
                   r=theta0[3])
    Tc = 3
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        AR.complex_step_grad(prm, Tc, np.zeros(2000), 1.0)
        tc = time.perf_counter() - t0
    return {"workload": "long_2000x20", "T": T, "K": K, "loss": loss,
            "grad": {"a": g[0], "A1": g[1], "A2": g[2], "r": g[3]},
            "forward_s": round(f, 4), "backward_s": round(b, 4),
            "backward_over_forward": round(b / f, 3),
            # gradient steps per second: steps of a run whose full gradient
            # (all four parameters) is had per second of forward + backward
            "gradient_steps_per_s": round(T / (f + b), 1),
            "cpu_oracle": {"value": round(Tc / tc, 3), "unit": "gradient steps per s", "cores": 1,
                           "kind": "oracle",
                           "sample": "complex-step gradient (four complex128 runs) of %d steps of the same "
                                     "channel, NumPy, one thread, %.1f s" % (Tc, tc)}}


def pressure_step(nx=4000, ny=40, steps=200000, spl=None):
    """The long pressure-driven channel of Section 3.2 (L/H = 100, 4000 x 40,
    p_in/p_out = 2, Kn_out = 0.1, linear-density start) run for its 2e5
    steps: time per step with HIP events on the solver's stream over the
    whole run, then the physics it is run for -- the non-linear centre-line
    pressure deviation dp(x) = (p_c - p_l)/p_out along the channel and the
    mass flow m = sum_y rho u_x (its column mean and its spread along x,
    which vanishes at steady state)."""
    import torch
    from paper_1603_01955_amd import Solver
    s = Solver(nx=nx, ny=ny, xbc="pressure", kn=0.1, p_ratio=2.0, init="linear_rho")
    if spl is not None:
        s.set_steps_per_launch(spl)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / steps
    dp, _ = s.pressure_deviation()
    m_col, m = s.massflow()
    dp = dp.cpu()
    m_col = m_col.cpu()
    ok = s.check_finite()
    s.close()
    k = int(torch.argmax(dp))
    at = [0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95]
    return {"workload": "pressure_%dx%d" % (nx, ny), "steps": steps, "us_per_step": round(us, 3),
            "mlups": round(nx * ny / us, 1), "finite": ok,
            "dp_max": round(float(dp[k]), 6), "x_over_L_at_dp_max": round((k + 0.5) / nx, 4),
            "dp_profile": {"x_over_L": at, "dp": [round(float(dp[min(nx - 1, int(a * nx))]), 6) for a in at]},
            "massflow_mean": float(m),
            "massflow_spread": float((m_col.max() - m_col.min()) / abs(m)),
            "cpu_oracle": pressure_oracle(nx, ny)}


def pressure_oracle(nx, ny):
    """The CPU reference on the same channel from the same start."""
    from oracle import clb_ref as C
    prm = C.Params(nx=nx, ny=ny, xbc="pressure", kn=0.1, p_ratio=2.0)
    st = {"P": C.init_linear_rho(prm)}

    def step():
        st["P"] = C.step(st["P"], prm)
    return oracle_rate(step, nx * ny, "the %dx%d channel" % (nx, ny))


def duct3d(steps=100, warmup=5):
    """The 3-D extension (rectangular microduct, D3Q27, 512 x 256 x 256,
    Kn = 0.5 of the height, g = 1e-6, seeded perturbed start): time per step
    with HIP events on the solver's stream; one step reads and writes every
    population once, 432 B per node update."""
    import torch
    from clb_inputs import WORKLOADS
    from paper_1603_01955_amd import Duct
    w = dict(WORKLOADS["duct_512x256x256"])
    s = Duct(**w)
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nodes = s.nx * s.ny * s.nz
    ok = s.check_finite()
    s.close()
    del s
    torch.cuda.empty_cache()
    gbs = 432.0 * nodes / (ms * 1e-3) / 1e9
    from oracle import clb3d_ref as D
    prm = D.Params3D(nx=w["nx"], ny=w["ny"], nz=w["nz"], kn=w["kn"], gx=w["gx"])
    win = {"P": D.init_perturbed_window(prm, w["seed"], w["init_amp"], 0, 8, 0, 8)}

    def step():
        win["P"] = D.run_window(win["P"], prm, 1)
    cpu = oracle_rate(step, w["nx"] * 64, "a 512 x 8 x 8 corner window of the same duct (the duct's rates)")
    return {"workload": "duct_512x256x256", "steps": steps, "ms_per_step": round(ms, 4), "finite": ok,
            "cpu_oracle": cpu,
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "unit_bytes": "432 B per node update"}}


def pressure_duct_steady(chunk=5000, max_chunks=40):
    """A shorter pressure-driven duct (400 x 8 x 8, p_in/p_out = 2,
    Kn_out = 0.1, linear start) run until its mass flow is the same through
    every cross-section to 1e-9: the axial pressure deviation of the steady
    state (its peak and where it lies) and the mass flow."""
    import numpy as np
    from paper_1603_01955_amd import Duct
    s = Duct(nx=400, ny=8, nz=8, xbc="pressure", kn=0.1, p_ratio=2.0, init="linear_rho")
    t0 = time.perf_counter()
    spread, mean, n = None, None, 0
    for _ in range(max_chunks):
        s.step(chunk)
        n += chunk
        m, mean = s.massflow()
        m = m.cpu().numpy()
        spread = float((m.max() - m.min()) / mean)
        if spread < 1e-9:
            break
    dp = s.pressure_deviation()[0].cpu().numpy()
    wall = time.perf_counter() - t0
    s.close()
    k = int(np.argmax(dp))
    return {"steps": n, "seconds": round(wall, 3), "mass_flow": mean, "mass_flow_spread": spread,
            "dp_max": round(float(dp[k]), 6), "x_over_L_at_dp_max": round((k + 0.5) / 400, 4)}


def duct3d_pressure(steps=200, warmup=5):
    """The pressure-driven 3-D duct (4000 x 40 x 40, L/H = 100,
    p_in/p_out = 2, Kn_out = 0.1, linear start): time per step with HIP
    events on the solver's stream.  A step is three launches: the two ghost
    planes, the rates of every cross-section, the step itself; the roofline
    unit is the step's 432 B per node update plus the ghost planes (54 values
    read and 27 written per row of each plane)."""
    import torch
    from clb_inputs import WORKLOADS
    from paper_1603_01955_amd import Duct
    w = dict(WORKLOADS["duct_pressure_4000x40x40"])
    s = Duct(**w)
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nodes = s.nx * s.ny * s.nz
    ok = s.check_finite()
    _, m_mean = s.massflow()
    s.close()
    del s
    torch.cuda.empty_cache()
    step_bytes = 432.0 * nodes + 2 * (54 + 27) * 8.0 * w["ny"] * w["nz"]
    gbs = step_bytes / (ms * 1e-3) / 1e9
    from oracle import clb3d_ref as D
    small = dict(nx=w["nx"], ny=4, nz=4, kn=w["kn"], xbc="pressure", p_ratio=w["p_ratio"])
    prm = D.Params3D(**small)
    st = {"P": D.init_linear_rho(prm)}

    def step():
        st["P"] = D.step(st["P"], prm)
    cpu = oracle_rate(step, w["nx"] * 16, "a 4000 x 4 x 4 pressure-driven duct (the same length, Kn_out and "
                                          "pressure ratio, the cross-section cut to 4 x 4)")
    steady = pressure_duct_steady()
    return {"workload": "duct_pressure_4000x40x40", "steps": steps, "ms_per_step": round(ms, 4), "finite": ok,
            "mass_flow_mean": m_mean, "steady_400x8x8": steady, "cpu_oracle": cpu,
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "unit_bytes": "432 B per node update + 648 B per row of each ghost plane"}}


def forcing_variant(steps=200, warmup=10):
    """The source with third-order force moments (clb_params.forcing = 1):
    the periodic step's throughput on the benchmark grid, and the batched Kn
    sweep's flow-rate minimum, which moves from 1/(sqrt(18 B2) - a) = 0.87 to
    the continuum 1/(sqrt(12 B2) - a) = 1.76 (no loop baselines)."""
    import torch
    from paper_1603_01955_amd import Solver
    s = Solver(forcing=1, **WORKLOAD)
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nodes = s.nx * s.ny
    s.close()
    del s
    torch.cuda.empty_cache()
    sw = kn_sweep(baselines=False, forcing=1)
    km = kn_minimum(forcing=1)
    return {"forcing": 1, "step_ms": round(ms, 4), "step_mlups": round(nodes / (ms * 1e-3) / 1e6, 1),
            "kn_sweep_all_converged": sw["all_converged"], "kn_sweep_batched_s": sw["batched_s"],
            "kn_minimum": km}


def mass_flow_sweep(check_every=2000, tol=1e-10, max_steps=3000000, step_probe=2000, baselines=True, spl=None):
    """Mass-flow study of Section 3.2: 16 long channels (2000 x 20, L/H = 100,
    p_in/p_out = 1.8, sigma = 0.93, Kn_out log-spaced 0.01-1, linear-density
    start) advanced together by the pressure batch, each to steady state
    (column-mean mass flow settled to tol over check_every steps).  Reports
    S = m / m_ns per channel, the batched step time against a loop of
    single-channel solvers, and the run to steady state against the same loop
    with the same checks."""
    import numpy as np
    import torch
    from clb_inputs import WORKLOADS, mass_flow_sweep_kn
    from paper_1603_01955_amd import PressureBatch, Solver, clb

    w = WORKLOADS["mass_flow_sweep_16x2000x20"]
    kns = mass_flow_sweep_kn(w["channels"], w["kn_lo"], w["kn_hi"])
    params = [clb.make_params(w["nx"], w["ny"], xbc="pressure", kn=k, p_ratio=w["p_ratio"], sigma=w["sigma"])
              for k in kns]
    nodes = w["channels"] * w["nx"] * w["ny"]

    def per_step_us(obj):
        obj.step(200)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(obj.stream)
        obj.step(step_probe)
        e1.record(obj.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / step_probe

    def batch():
        b = PressureBatch(params)
        if spl is not None:
            b.set_steps_per_launch(spl)
        return b

    def single(p):
        one = Solver(params=p)
        if spl is not None:
            one.set_steps_per_launch(spl)
        return one

    pb = batch()
    us_batch = per_step_us(pb)
    pb.close()
    pb = batch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_b, conv = pb.run(max_steps, check_every, tol)        # synchronises
    t_batch = time.perf_counter() - t0
    m, m_ns = pb.massflow()
    pb.close()
    out = {"workload": "mass_flow_sweep_16x2000x20", "channels": len(params), "p_ratio": w["p_ratio"],
           "sigma": w["sigma"], "kn_out": [round(k, 5) for k in kns],
           # Kn_ave = (Kn_in + Kn_out) / 2, Kn_in = Kn_out p_out / p_in (the abscissa of the
           # S plot of the mass-flow study, Section 3.2); 1/S is the other plot's ordinate
           "kn_ave": [round(k * (1.0 + 1.0 / w["p_ratio"]) / 2.0, 5) for k in kns],
           "S": [round(float(v), 6) for v in m / m_ns],
           "inv_S": [round(float(v), 6) for v in m_ns / m], "all_converged": bool(conv.all()),
           "steps": [int(v) for v in steps_b], "check_every": check_every, "tol": tol,
           "batched_to_steady_s": round(t_batch, 3),
           "batched_step_us": round(us_batch, 3), "batched_mlups": round(nodes / us_batch, 1),
           "batched_algorithmic_gbs": round(BYTES_PER_NODE * nodes / us_batch / 1e3, 1)}
    from oracle import clb_ref as C
    prm0 = C.Params(nx=w["nx"], ny=w["ny"], xbc="pressure", kn=kns[0], p_ratio=w["p_ratio"], sigma=w["sigma"])
    st = {"P": C.init_linear_rho(prm0)}

    def ostep():
        st["P"] = C.step(st["P"], prm0)
    out["cpu_oracle"] = oracle_rate(ostep, w["nx"] * w["ny"], "one channel of the batch (the first; the reference "
                                    "steps channels one at a time)")
    if not baselines:
        return out
    s = single(params[0])
    s.set_graph_steps(step_probe // 10)
    us_single = per_step_us(s)
    s.close()
    out["loop_step_us"] = round(us_single * len(params), 3)
    out["step_speedup_vs_graph_loop"] = round(us_single * len(params) / us_batch, 2)
    torch.cuda.synchronize()
    steps_l = []
    t0 = time.perf_counter()
    for p in params:
        s = single(p)
        s.set_graph_steps(check_every)
        prev, n = float("nan"), 0
        while n < max_steps:
            s.step(check_every)
            n += check_every
            cur = s.massflow()[1]                              # synchronises
            if abs(cur - prev) <= tol * abs(cur):
                break
            prev = cur
        steps_l.append(n)
        s.close()
    t_loop = time.perf_counter() - t0
    out["graph_loop_to_steady_s"] = round(t_loop, 3)
    out["loop_steps_match"] = bool((np.array(steps_l) == steps_b).all())
    out["speedup_vs_graph_loop"] = round(t_loop / t_batch, 2)
    return out


def oracle_rate(step, nodes, sample, budget_s=3.0):
    """The CPU reference as it stands, one thread, timed beside a GPU row:
    step() advances its state by one step of `nodes` node updates; steps
    are taken (after one warm-up step) until budget_s has passed."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        step()
        n = 0
        t0 = time.perf_counter()
        while True:
            step()
            n += 1
            dt = time.perf_counter() - t0
            if dt >= budget_s:
                break
    return {"value": round(nodes * n / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%d steps of %s, NumPy FP64, one thread, %.1f s" % (n, sample, dt)}


def cpu_baseline():
    """The CPU reference, as it stands, on a bounded sample of the workload:
    CPU_SAMPLE_STEPS steps of a CPU_SAMPLE_NX x 2048 slab of the same channel
    (full height, so the wall rows are 2 of 2048 as on the full grid; same Kn,
    force and seeded start; periodic over the slab), BLAS and OpenMP pools
    limited to one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import clb_ref as C
    prm = C.Params(nx=CPU_SAMPLE_NX, ny=WORKLOAD["ny"], kn=WORKLOAD["kn"], gx=WORKLOAD["gx"])
    with threadpool_limits(limits=1):
        P = C.init_perturbed(prm, WORKLOAD["seed"], WORKLOAD["init_amp"])
        P = C.step(P, prm)                      # warm-up
        t0 = time.perf_counter()
        P = C.run(P, prm, CPU_SAMPLE_STEPS)
        dt = time.perf_counter() - t0
    nodes = prm.nx * prm.ny
    return {"value": nodes * CPU_SAMPLE_STEPS / dt / 1e6, "unit": "MLUPS", "cores": 1,
            "kind": "oracle", "host_cores": os.cpu_count(),
            "thread_pins": {"threadpool_limits": 1, "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
                            "OPENBLAS_NUM_THREADS": os.environ.get("OPENBLAS_NUM_THREADS")},
            "sample": "%d steps of a %dx%d slab of the same channel (full height; Kn=1, g=1e-7, seeded start), "
                      "NumPy FP64, one thread, %.1f s" % (CPU_SAMPLE_STEPS, prm.nx, prm.ny, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.part == "sweep":
        print(json.dumps({"kn_sweep": kn_sweep(baselines=not args.no_loop_baseline),
                          "kn_minimum": kn_minimum()}), flush=True)
        return
    if args.part == "pressure":
        print(json.dumps({"pressure_step": pressure_step(steps=args.pressure_steps,
                                                         spl=args.channel_steps_per_launch)}), flush=True)
        return
    if args.part == "msweep":
        print(json.dumps({"mass_flow_sweep": mass_flow_sweep(max_steps=args.msweep_max_steps,
                                                             baselines=not args.no_loop_baseline,
                                                             spl=args.channel_steps_per_launch)}), flush=True)
        return
    if args.part == "adjoint":
        print(json.dumps({"adjoint": adjoint_calibration()}), flush=True)
        return
    if args.part == "duct":
        print(json.dumps({"duct3d": duct3d()}), flush=True)
        return
    if args.part == "pduct":
        print(json.dumps({"duct3d_pressure": duct3d_pressure()}), flush=True)
        return
    import torch
    from paper_1603_01955_amd import Solver

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = Solver(device=dev, **WORKLOAD)
    s.set_launch(args.block_x, args.xcd_remap)
    s.set_steps_per_launch(args.steps_per_launch)
    nodes = s.nx * s.ny
    s.step(args.warmup)
    torch.cuda.synchronize()
    stream = s.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    s.step(args.steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    ok = s.check_finite()
    mlups = nodes / (ms * 1e-3) / 1e6
    k = args.steps_per_launch if s.nx >= 64 else 1   # narrower grids step one at a time
    def at_steps_per_launch(kk, n):
        """The same grid at kk steps per launch: its speed and its launch's
        HBM fraction (144 B per node per launch over the launch time)."""
        s.set_steps_per_launch(kk)
        s.step(2 * kk)
        n = max(kk, n // kk * kk)
        t0.record(stream)
        s.step(n)
        t1.record(stream)
        torch.cuda.synchronize()
        msk = t0.elapsed_time(t1) / n
        gbs = BYTES_PER_NODE * nodes / (kk * msk * 1e-3) / 1e9
        return {"steps_per_launch": kk, "steps": n, "ms_per_step": round(msk, 4),
                "mlups": round(nodes / (msk * 1e-3) / 1e6, 1), "achieved": round(gbs, 1),
                "frac": round(gbs / HBM_PEAK_GBS, 4)}

    # the same grid at two steps per launch and at one (the one-step kernel),
    # for their HBM fractions: fewer steps per launch draw more of HBM and
    # advance the grid more slowly
    alt = alt1 = None
    if s.nx >= 64 and args.part != "step":   # the step part times the default form alone (profiling runs)
        if k != 2:
            alt = at_steps_per_launch(2, args.steps)
        if k != 1:
            alt1 = at_steps_per_launch(1, min(args.steps, 300))
    # average duration of one k-step launch (steps % k of the timed steps run
    # in one shorter launch at the end: one launch in 334 at 1000 steps, k = 3)
    launch_s = ms * 1e-3 * k
    # Algorithmic bytes of one k-step launch: every population read once and
    # written once (72 B + 72 B per node); the steps before the last stay in LDS.
    alg = BYTES_PER_NODE * nodes
    achieved = alg / launch_s / 1e9
    prof = profile_record()
    traffic = float(prof["bytes_per_launch"]) if "bytes_per_launch" in prof and int(
        prof.get("steps_per_launch", 0)) == k else None
    fp64 = float(prof["fp64_valu_insts_per_launch"]) if "fp64_valu_insts_per_launch" in prof and int(
        prof.get("steps_per_launch", 0)) == k else None
    valu = float(prof["valu_insts_per_launch"]) if "valu_insts_per_launch" in prof and int(
        prof.get("steps_per_launch", 0)) == k else None
    copy_gbs = copy_bandwidth()
    # Lower bounds on the launch time: its counted HBM bytes at the copy rate
    # measured above, and its counted VALU instructions at one wave
    # instruction per CU per clock.  The larger one over the measured time is
    # how close the launch runs to what binds it.
    t_hbm = traffic / (copy_gbs * 1e9) if traffic else None
    t_valu = valu / FP64_WAVE_INSTS_PER_S if valu else None
    rec = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "periodic_32768x2048", "nx": s.nx, "ny": s.ny, "kn": WORKLOAD["kn"],
                   "g": WORKLOAD["gx"], "start": "seeded perturbed equilibrium, amp 1e-4, seed 12345",
                   "buffers": "A-B", "block_x": args.block_x, "xcd_remap": args.xcd_remap,
                   "steps_per_launch": k},
        "finite": ok,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "steps_per_launch": k,
                     "launch_us": round(launch_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": alg,
                     "unit_bytes": "144 B per node per launch (9 FP64 read + 9 written once; "
                                   "a launch advances every node k steps)",
                     # the HBM ceiling measured on this GPU
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4),
                     # counter bytes per launch over the launch time: the bandwidth actually drawn
                     "traffic_gbs": round(traffic / launch_s / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                     # FP64 VALU instructions per launch (counters) against one per clock per CU
                     "fp64_issue_frac": round(fp64 / launch_s / FP64_WAVE_INSTS_PER_S, 4) if fp64 else None,
                     # node updates x 144 B over the time: the bandwidth a one-step kernel would need
                     "effective_gbs": round(BYTES_PER_NODE * nodes * k / launch_s / 1e9, 1),
                     "two_steps_per_launch": alt,
                     "one_step_per_launch": alt1,
                     "bound_us": {"hbm_at_copy_rate": round(t_hbm * 1e6, 1) if t_hbm else None,
                                  "valu_issue": round(t_valu * 1e6, 1) if t_valu else None},
                     "bound_time_frac": round(max(t_hbm, t_valu) / launch_s, 4) if t_hbm and t_valu else None},
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    if args.part == "step":
        print(json.dumps(rec), flush=True)
        return
    if not args.no_sweep:
        rec["kn_sweep"] = kn_sweep(baselines=not args.no_loop_baseline)
        rec["kn_minimum"] = kn_minimum()
    rec["pressure_step"] = pressure_step()
    rec["forcing_variant"] = forcing_variant()
    if not args.no_msweep:
        rec["mass_flow_sweep"] = mass_flow_sweep(max_steps=args.msweep_max_steps,
                                                 baselines=not args.no_loop_baseline)
    if not args.no_adjoint:
        rec["adjoint"] = adjoint_calibration()
    rec["duct3d"] = duct3d()
    rec["duct3d_pressure"] = duct3d_pressure()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
