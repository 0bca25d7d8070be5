"""Why the kernels divide by 3 (and 6) through a split constant.

The collision at tau = 1/2 is f* = 2 f^eq - f, and every 2 f^eq is a field
combination times 1/3.  Summed over the populations of a cell it returns
the moments D and B unchanged (section 2.1: the collision conserves them).
With the FP32-rounded 1/3 (3.0e-8 too large) the sum is 2 (1 + 3e-8) D - D,
so the moments gain 6e-8 per step, systematically; a wave that has
travelled T steps is too strong by ~6e-8 T (1e-4 after the ~1500 steps a
wave takes across a 1024^2 grid).  Splitting the constant into its rounded
head and tail, x/3 = fma(x, head, x * tail), rounds x/3 correctly, and the
remaining rounding errors carry no bias.  The kernels divide the fields
once per cell this way and form each population's combination from the
thirds.

Checked here on a float32 emulation of the reduced 2-D TM update (the
eleven scalars of the kernels, a periodic row carrying a vacuum plane
wave from its equilibrium) against the same update in float64.
"""
import numpy as np
import pytest

F32 = np.float32


def _r(x):
    return np.asarray(x, np.float64).astype(np.float32)


def _fma(a, b, c):
    # single rounding: the float32 x float32 product is exact in float64
    return (np.float64(a) * np.float64(b) + np.float64(c)).astype(np.float32)


def _run(steps, mode, n=64, lam=32.0):
    x = np.arange(n)
    E = np.sin(2 * np.pi * x / lam)
    H = -E                                     # +x propagation: H = xhat x E
    Ez, Hx, Hy = E, np.zeros(n), H
    f = np.array([Ez - Hy, Ez + Hy, Ez + Hx, Ez - Hx, Hx, Hx, Hy, Hy, Ez, Hx, Hy]) / 6.0
    if mode != "f64":
        f = f.astype(np.float32)
    hi = np.float32(1.0 / 3.0)
    lo = np.float32(1.0 / 3.0 - np.float64(hi))
    for _ in range(steps):
        g = f.copy()
        g[0], g[4] = np.roll(f[0], 1), np.roll(f[4], 1)      # +x movers from x - 1
        g[1], g[5] = np.roll(f[1], -1), np.roll(f[5], -1)    # -x movers from x + 1
        if mode == "f64":
            Ez = 2 * g[8] + g[0] + g[1] + g[2] + g[3]
            Hx = 2 * g[9] + g[4] + g[5] + g[2] - g[3]
            Hy = 2 * g[10] + g[6] + g[7] - g[0] + g[1]
            X = [Ez - Hy, Ez + Hy, Ez + Hx, Ez - Hx, Hx, Hx, Hy, Hy, Ez, Hx, Hy]
            f = np.array([X[i] / 3.0 - g[i] for i in range(11)])
            continue
        Ez = _fma(F32(2), g[8], _r(_r(_r(g[0] + g[1]) + g[2]) + g[3]))
        Hx = _fma(F32(2), g[9], _r(_r(_r(g[4] + g[5]) + g[2]) - g[3]))
        Hy = _fma(F32(2), g[10], _r(_r(_r(g[6] + g[7]) - g[0]) + g[1]))
        X = [_r(Ez - Hy), _r(Ez + Hy), _r(Ez + Hx), _r(Ez - Hx), Hx, Hx, Hy, Hy, Ez, Hx, Hy]
        if mode == "rounded":                  # fma(fl(1/3), X, -f)
            f = np.array([_fma(hi, X[i], -g[i]) for i in range(11)])
        else:                                  # fields/3 by the split constant, then combined
            t3 = lambda v: _fma(hi, v, _r(np.float64(v) * np.float64(lo)))
            ez, hx, hy = t3(Ez), t3(Hx), t3(Hy)
            Y = [_r(ez - hy), _r(ez + hy), _r(ez + hx), _r(ez - hx), hx, hx, hy, hy, ez, hx, hy]
            f = np.array([_r(np.float64(Y[i]) - np.float64(g[i])) for i in range(11)])
    return (2 * f[8].astype(np.float64) + f[0] + f[1] + f[2] + f[3])


@pytest.mark.parametrize("steps", [1500])
def test_split_third_removes_the_fp32_gain(steps):
    ref = _run(steps, "f64")
    amp = lambda e: float(np.sqrt(np.sum(e ** 2) / np.sum(ref ** 2)))
    err = lambda e: float(np.sqrt(np.sum((e - ref) ** 2) / np.sum(ref ** 2)))
    rounded, split = _run(steps, "rounded"), _run(steps, "split")
    # the rounded constant: a gain of ~6e-8 per step
    assert 0.8 * 6e-8 * steps < amp(rounded) - 1.0 < 1.2 * 6e-8 * steps
    # the split constant: no systematic gain, 20x smaller error
    assert abs(amp(split) - 1.0) < 1e-5
    assert err(split) < err(rounded) / 20
