"""Pins of the oracle's discrete adjoint (inverse design, far-field
objective): central finite differences in FP64 on a tiny grid."""
import numpy as np

import workloads as W
from oracle.adjoint import FarFieldObjective


def _tiny_case():
    n = 40
    case = W.cylinder_case(2.25, "TM", n=n, a=4.0, lam=8.0, W=8, steps=260, half=9.5)
    rng = np.random.default_rng(7)
    eps = np.ones((1, n, n))
    eps[0, 16:24, 16:24] = rng.uniform(1.0, 4.0, (8, 8))
    case.eps = eps
    return case


def test_adjoint_gradient_matches_central_differences():
    case = _tiny_case()
    obj = FarFieldObjective(case, np.arange(10.0, 20.01, 0.5), sigma_max=W.SIGMA_MAX,
                            ramp_periods=1.0)
    J, grad = obj.value_and_gradient(case.eps)
    assert J > 0
    rng = np.random.default_rng(2510)
    h = 1e-5
    for _ in range(5):
        y, x = rng.integers(16, 24, 2)
        ep, em = case.eps.copy(), case.eps.copy()
        ep[0, y, x] += h
        em[0, y, x] -= h
        fd = (obj.value(ep) - obj.value(em)) / (2 * h)
        assert abs(grad[0, y, x] - fd) <= 1e-6 * np.abs(grad).max() + 1e-7 * abs(fd), (y, x, grad[0, y, x], fd)
    # cells outside the design region still get a gradient (eps = 1 there):
    # the adjoint is a full-field sensitivity; the design region is a subset
    assert np.abs(grad[0, 16:24, 16:24]).max() > 0
