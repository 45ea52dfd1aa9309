"""GPU tests of the hand-written adjoint of the pressure-driven run, through
the C ABI: one reverse step against complex-step Jacobian products of the CPU
reference (dot-product test), whole-run gradients against the reference's
complex-step gradients, invariance to the checkpoint interval, central finite
differences at the long-channel size, and the autograd entry point."""
import dataclasses

import numpy as np
import pytest
import torch

from clb_inputs import uniform_populations
from oracle import adjoint_ref as R
from oracle import clb_ref as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")


def _gpu_params(prm, r_free=True):
    from paper_1603_01955_amd import clb
    A1, r = C.resolved(prm)
    return clb.make_params(prm.nx, prm.ny, xbc="pressure", kn=prm.kn, p_ratio=prm.p_ratio, a=prm.a,
                           A1=A1, A2=prm.A2, r=r if r_free else None, sigma=prm.sigma,
                           cbbsr_shift=prm.cbbsr_shift, tq_den=prm.tq_den, rho_out=prm.rho_out)


def _adjoint(prm, T, K, r_free=True):
    from paper_1603_01955_amd.adjoint import Adjoint
    return Adjoint(_gpu_params(prm, r_free), T, K)


@pytest.mark.parametrize("nx,ny,shift,extra", [(48, 6, 1, {}), (130, 5, 1, {}), (20, 2, 1, {}), (33, 4, 0, {}),
                                               (2, 3, 1, {}),
                                               (40, 7, 1, dict(tq_den=24.0, A2=0.3, sigma=0.8, rho_out=1.2))])
def test_vjp_step_dot_product(nx, ny, shift, extra):
    """<lambda, J v> (J v by complex step of the reference step) equals
    <J^T lambda, v> from the GPU reverse step; same for the parameters."""
    prm = C.Params(nx=nx, ny=ny, xbc="pressure", kn=0.2, p_ratio=1.7, cbbsr_shift=shift, **extra)
    A1, r = C.resolved(prm)
    prm = dataclasses.replace(prm, A1=A1, r=r)
    P = C.init_linear_rho(prm) + uniform_populations(nx, ny, seed=31, lo=-5e-3, hi=5e-3)
    lam = uniform_populations(nx, ny, seed=32, lo=-1.0, hi=1.0)
    v = uniform_populations(nx, ny, seed=33, lo=-1.0, hi=1.0)
    h = 1e-30
    Jv = np.imag(C.step(P + 1j * h * v, prm)) / h
    adj = _adjoint(prm, 1, 1)
    lam_prev, g3 = adj.vjp_step(torch.from_numpy(P), torch.from_numpy(lam))
    lam_prev = lam_prev.cpu().numpy()
    lhs, rhs = float(np.sum(lam * Jv)), float(np.sum(lam_prev * v))
    assert abs(lhs - rhs) <= 1e-11 * np.sum(np.abs(lam * Jv))
    for k, name in enumerate(("a", "A2", "r")):
        q = dataclasses.replace(prm, **{name: getattr(prm, name) + 1j * h})
        dstep = np.imag(C.step(P.astype(np.complex128), q)) / h
        ref = float(np.sum(lam * dstep))
        assert abs(g3[k] - ref) <= 1e-10 * np.sum(np.abs(lam * dstep)) + 1e-300, name


def _case(nx=64, ny=6, T=60):
    prm = C.Params(nx=nx, ny=ny, xbc="pressure", kn=0.1, p_ratio=2.0)
    tgt = dataclasses.replace(prm, a=2.1, A2=0.52, r=0.64)
    dps, ms = R.observables(R.run(tgt, T), tgt)
    return prm, dps, ms


@pytest.mark.parametrize("r_free", [True, False])
def test_gradient_matches_complex_step(r_free):
    T = 60
    prm, dps, ms = _case(T=T)
    A1, r = C.resolved(prm)
    ref_prm = dataclasses.replace(prm, A1=A1, r=r if r_free else None)
    ref = R.complex_step_grad(ref_prm, T, dps, ms)
    L_ref = R.loss(ref_prm, T, dps, ms)
    adj = _adjoint(prm, T, 8, r_free)
    L = adj.forward(torch.from_numpy(dps), ms)
    assert abs(L - L_ref) <= 1e-10 * abs(L_ref)
    dp, m = adj.observables()
    assert np.max(np.abs(dp.cpu().numpy() - R.observables(R.run(ref_prm, T), ref_prm)[0])) <= 1e-10
    g = adj.backward()
    want = np.array([ref["a"], ref["A1"], ref["A2"], ref["r"] if r_free else ref["r"]])
    if r_free:
        want[1] = 0.0
    scale = np.max(np.abs(want))
    assert np.max(np.abs(g[[0, 2, 3]] - want[[0, 2, 3]])) <= 1e-9 * scale
    assert abs(g[1] - want[1]) <= 1e-9 * scale


@pytest.mark.parametrize("nx,ny,T,K,shift", [
    (49, 6, 30, 7, 1),     # 16-column workgroups, nx = 1 (mod 16): column nx - 2 in the second-to-last one
    (50, 6, 30, 7, 1),     # column nx - 2 opens the last workgroup
    (9, 70, 12, 4, 1),     # ny > 64: several rows per thread, nx = 1 (mod 4)
    (17, 33, 16, 5, 0),    # odd ny, 4-column workgroups, literal Eq. (20) source
])
def test_gradient_workgroup_edges(nx, ny, T, K, shift):
    """Whole-run gradients where the inlet/outlet columns fall across
    workgroup boundaries of the reverse step, against complex-step."""
    prm = C.Params(nx=nx, ny=ny, xbc="pressure", kn=0.15, p_ratio=1.8, cbbsr_shift=shift)
    tgt = dataclasses.replace(prm, a=2.1, A2=0.52, r=0.64)
    dps, ms = R.observables(R.run(tgt, T), tgt)
    A1, r = C.resolved(prm)
    ref_prm = dataclasses.replace(prm, A1=A1, r=r)
    ref = R.complex_step_grad(ref_prm, T, dps, ms)
    adj = _adjoint(prm, T, K)
    L = adj.forward(torch.from_numpy(dps), ms)
    assert abs(L - R.loss(ref_prm, T, dps, ms)) <= 1e-10 * abs(L)
    g = adj.backward()
    want = np.array([ref["a"], ref["A2"], ref["r"]])
    assert np.max(np.abs(g[[0, 2, 3]] - want)) <= 1e-9 * np.max(np.abs(want))
    assert g[1] == 0.0


def test_checkpoint_interval_does_not_change_gradients():
    T = 37
    prm, dps, ms = _case(nx=40, ny=5, T=T)
    grads = []
    for K in (1, 6, 37):
        adj = _adjoint(prm, T, K)
        adj.forward(torch.from_numpy(dps), ms)
        grads.append(adj.backward())
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])


def test_gradient_vs_central_differences_long_channel():
    """Long channel L/H = 100, 2000 x 20, pressure ratio 2, Kn_out = 0.1,
    T = 2000 steps with 45-step checkpoints; target from the same run with
    perturbed (a, A2, r); central differences with h = 1e-6 |theta|."""
    from paper_1603_01955_amd import clb
    from paper_1603_01955_amd.adjoint import Adjoint
    T, K = 2000, 45
    base = dict(xbc="pressure", kn=0.1, p_ratio=2.0)
    theta = np.array([2.0, 0.0, 0.55, C.bounce_fraction(C.slip_A1(1.0))])

    def params(th):
        return clb.make_params(2000, 20, a=th[0], A2=th[2], r=th[3], **base)

    star = theta * np.array([1.04, 1.0, 0.93, 1.03])
    tgt = Adjoint(params(star), T, K)
    tgt.forward(torch.zeros(2000, dtype=torch.float64), 1.0)
    dps, ms = tgt.observables()
    tgt.close()
    adj = Adjoint(params(theta), T, K)
    adj.forward(dps, ms)
    g = adj.backward()

    def L(th):
        a = Adjoint(params(th), T, K)
        v = a.forward(dps, ms)
        a.close()
        return v

    for k in (0, 2, 3):
        h = 1e-6 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(g[k] - fd) <= 1e-6 * abs(g[k]), (k, g[k], fd)


def test_autograd_function():
    from paper_1603_01955_amd.adjoint import CLBRunLoss
    T = 30
    prm, dps, ms = _case(nx=40, ny=6, T=T)
    A1, r = C.resolved(prm)
    theta = torch.tensor([prm.a, A1, prm.A2, r], dtype=torch.float64, requires_grad=True)
    spec = dict(nx=40, ny=6, kn=prm.kn, p_ratio=prm.p_ratio, T=T, K=6, dp_target=dps, m_target=ms,
                r_free=True)
    loss = CLBRunLoss.apply(theta, spec)
    loss.backward()
    ref = R.complex_step_grad(dataclasses.replace(prm, A1=A1, r=r), T, dps, ms)
    want = torch.tensor([ref["a"], 0.0, ref["A2"], ref["r"]], dtype=torch.float64)
    assert torch.allclose(theta.grad, want, rtol=1e-9, atol=1e-9 * float(want.abs().max()))


def test_large_grid_forward_takes_row_kernel():
    """8192 x 256 (2 M nodes): the adjoint's forward steps take the row
    kernel; its final observables equal a column-kernel solver's bit for bit,
    and the backward sweep runs at this size with finite gradients."""
    from paper_1603_01955_amd import Solver, clb
    from paper_1603_01955_amd.adjoint import Adjoint
    nx, ny, T = 8192, 256, 3
    p = clb.make_params(nx, ny, xbc="pressure", kn=0.2, p_ratio=1.5)
    adj = Adjoint(p, T, 2)
    adj.forward(torch.zeros(nx, dtype=torch.float64), 1.0)
    dp, m = adj.observables()
    s = Solver(params=clb.make_params(nx, ny, xbc="pressure", kn=0.2, p_ratio=1.5, init="linear_rho"))
    s.set_pressure_path(1)
    s.step(T)
    dp_ref, _ = s.pressure_deviation()
    assert torch.equal(dp.cpu(), dp_ref.cpu())
    assert m == s.massflow()[0][-1].item()
    g = adj.backward()
    assert np.all(np.isfinite(g))
    s.close()
    adj.close()
