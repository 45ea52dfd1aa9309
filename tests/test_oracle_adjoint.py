"""Pins of the reference gradient (complex-step differentiation of the CPU
reference run, Section 3.2 loss) against central finite differences of the
real-valued reference and the chain rule of Eq. (21)."""
import dataclasses
from math import pi, sqrt

import pytest

from oracle import adjoint_ref as R
from oracle import clb_ref as C


@pytest.fixture(scope="module")
def case():
    prm = C.Params(nx=24, ny=5, xbc="pressure", kn=0.15, p_ratio=1.8)
    tgt = dataclasses.replace(prm, a=2.1, A2=0.5, r=0.6)
    P = R.run(tgt, 16)
    dps, ms = R.observables(P, tgt)
    return prm, dps, ms


@pytest.mark.parametrize("name", ["a", "A1", "A2", "r"])
def test_complex_step_matches_central_differences(case, name):
    prm, dps, ms = case
    g = R.complex_step_grad(prm, 16, dps, ms, names=(name,))[name]
    A1, r = C.resolved(prm)
    base = {"A1": A1, "r": r}.get(name, getattr(prm, name))
    h = 1e-6 * abs(base)

    def L(v):
        kw = {name: v}
        if name == "r":
            kw["A1"] = A1
        if name == "A1":
            kw["r"] = None
        return R.loss(dataclasses.replace(prm, **kw), 16, dps, ms)

    fd = (L(base + h) - L(base - h)) / (2 * h)
    assert abs(g - fd) <= 1e-6 * abs(g)


def test_A1_acts_only_through_r(case):
    prm, dps, ms = case
    g = R.complex_step_grad(prm, 16, dps, ms, names=("A1", "r"))
    _, r = C.resolved(prm)
    assert g["A1"] == pytest.approx(g["r"] * (-sqrt(pi / 6.0) * r * r), rel=1e-10)
    pr = dataclasses.replace(prm, r=r)
    assert R.complex_step_grad(pr, 16, dps, ms, names=("A1",))["A1"] == 0.0
