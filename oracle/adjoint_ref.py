"""Reference loss and gradients of the pressure-driven run (test infrastructure).

The loss of a run of T steps from the linear-density start (Section 3.2):
  L = (1/nx) sum_x (dp(x) - dp*(x))^2 + ((m - m*)/m*)^2,
dp the centre-line pressure deviation and m = sum_y rho u_x at the outlet
column of the state after T steps.  Gradients by complex-step
differentiation (Squire & Trapp, SIAM Review 40, 1998): the reference is run
in complex128 with one parameter shifted by i h, and dL/dtheta = Im L / h,
exact to rounding for h ~ 1e-30 because no subtraction is involved.
"""
import dataclasses

import numpy as np

from . import clb_ref as C


def observables(P, prm):
    """(dp(x), m at the outlet column) of the state P."""
    dp = C.pressure_deviation(P, prm)
    m = C.column_sums(P, prm)[0][-1]
    return dp, m


def run(prm, T, dtype=np.float64):
    P = C.init_linear_rho(prm, dtype=dtype)
    return C.run(P, prm, T)


def loss(prm, T, dp_target, m_target, dtype=np.float64):
    P = run(prm, T, dtype)
    dp, m = observables(P, prm)
    q = (m - m_target) / m_target
    return np.mean((dp - dp_target) ** 2) + q * q


def complex_step_grad(prm, T, dp_target, m_target, names=("a", "A1", "A2", "r"), h=1e-30):
    """dL/dtheta for each named parameter.  'A1' moves r through Eq. (21)
    unless prm.r is set; 'r' treats the bounce-back fraction as independent
    (taken from A1 when prm.r is None)."""
    A1, r = C.resolved(prm)
    out = {}
    for name in names:
        if name == "A1":
            if prm.r is not None:
                out[name] = 0.0
                continue
            q = dataclasses.replace(prm, A1=A1 + 1j * h, r=None)
        elif name == "r":
            q = dataclasses.replace(prm, A1=A1, r=r + 1j * h)
        else:
            q = dataclasses.replace(prm, **{name: getattr(prm, name) + 1j * h})
        out[name] = float(np.imag(loss(q, T, dp_target, m_target, dtype=np.complex128)) / h)
    return out
