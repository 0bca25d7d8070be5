"""The allocation-free far field (lbm_em_farfield_static) through the C ABI
against lbm_em_farfield on the same handles: two calls in a row, the second
with fewer angles; 2-D with a companion run, 2-D with the incident line, 3-D
with a companion run.  Both entry points run the same far-field arithmetic,
so the bar is the FP64 one (1e-12 relative to the largest |S|^2)."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_11042_amd as P

    return P


def _call(P, name, sim, inc, th, ph):
    from paper_2510_11042_amd import _lib

    out = np.full(th.size, np.nan)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    th = np.ascontiguousarray(th, dtype=np.float64)
    php = None if ph is None else dp(np.ascontiguousarray(ph, dtype=np.float64))
    st = getattr(_lib.lib(), name)(sim.handle, inc.handle if inc is not None else None, dp(th), php, th.size,
                                   dp(out))
    _lib.check(st)
    return out


def _compare(P, sim, inc, th_list, ph_list, tag):
    for th, ph in zip(th_list, ph_list):
        ref = _call(P, "lbm_em_farfield", sim, inc, th, ph)
        got = _call(P, "lbm_em_farfield_static", sim, inc, th, ph)
        err = np.abs(got - ref).max() / ref.max()
        say(tag, th.size, "max rel err", err)
        assert np.all(np.isfinite(got)) and err <= 1e-12


def _cyl(P, case, line=False):
    kh, eh = W.plane_wave_2d(case.theta_deg, case.pol)
    s = P.Simulation(case.nx, case.ny, 1, pol=case.pol, precision="fp32", absorb=case.absorb,
                     sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
    s.set_ntff(case.box_lo, case.box_hi, *case.window)
    if line:
        s.set_incident_line(True)
    s.step(case.steps)
    return s


def test_farfield_static_matches_farfield_2d(P):
    case = W.cylinder_case(2.25, "TE", n=192, a=10.5, lam=32.0, W=32, steps=1200, half=19.5)
    tot = _cyl(P, case)
    inc = _cyl(P, W.vacuum_companion(case))
    big = np.arange(0.0, 360.0, 0.25)
    small = np.linspace(3.0, 177.0, 97)
    _compare(P, tot, inc, [big, small], [None, None], "2-D companion")
    line = _cyl(P, case, line=True)
    _compare(P, line, None, [big, small], [None, None], "2-D line")
    for s in (tot, inc, line):
        s.close()


def test_farfield_static_matches_farfield_3d(P):
    n = 48
    case = W.sphere_case(n=n, x_size=2.5, lam=12.0, eps_in=2.25, W=8, steps=360, half=8.5)
    sims = []
    for eps in (case.eps, np.ones_like(case.eps)):
        s = P.Simulation(n, n, n, pol="3D", precision="fp32", absorb=(8, 8, 8), sigma_max=W.SIGMA_MAX)
        s.set_permittivity(eps)
        s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, 1.0)
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
        s.step(case.steps)
        sims.append(s)
    th = np.tile(np.arange(0.0, 180.01, 0.5), 3)
    ph = np.repeat([0.0, 45.0, 90.0], 361)
    _compare(P, sims[0], sims[1], [th, th[:50]], [ph, ph[:50] + 10.0], "3-D companion")
    for s in sims:
        s.close()


def test_farfield_static_limits(P):
    from paper_2510_11042_amd import LbmEmError

    case = W.cylinder_case(2.25, "TM", n=96, a=6.0, lam=16.0, W=16, steps=300, half=12.5)
    s = _cyl(P, case)
    too_many = np.zeros(4097)
    with pytest.raises(LbmEmError, match="MAX_ANGLES"):
        _call(P, "lbm_em_farfield_static", s, None, too_many, None)
    ok = np.arange(0.0, 360.0, 360.0 / 4096)
    assert ok.size == 4096
    out = _call(P, "lbm_em_farfield_static", s, None, ok, None)
    assert np.all(np.isfinite(out))
    s.close()
