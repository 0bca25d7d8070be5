"""The paper's own resolutions, rerun on the GPU and scored like the paper.

Section 3.2 (Table cylinder_RMS_combined, Table
cylinder_simulation_parameters) and section 3.4 (Table sphere_RMS, Table
dielectric_sphere_er_2) give, per case, L/a, a/dx and lambda/dx (or
lambda_eps/dx) and the normalised RMS error of |S|^2 against Lorenz-Mie
(Eq. rms_error).  Each case here uses those resolutions and domain sizes
(plus this implementation's absorbing layer around the domain), runs until
two consecutive one-period DFT windows agree, and is scored at 0.5 degree
sampling over 0..180 degrees.

Measured here (FP32) vs the paper's value:
  cylinder eps 2, a/lambda = 1     8.2e-4   (7.8e-4)
  cylinder eps 2, a/lambda = 0.1   3.8e-3   (8.4e-3)
  cylinder eps 2, a/lambda = 10    2.6e-3   (1.3e-3)
  cylinder a/lambda = 1, eps 5     1.5e-3   (1.0e-3)
  cylinder a/lambda = 1, eps 10    2.5e-3   (2.3e-3)
  cylinder a/lambda = 1, eps 20    2.5e-2   (6.6e-3)  -- converged, 3.7x the paper's error (a 4x thicker
                                   layer changes it only to 2.2e-2); bound 3e-2 guards it.  At m = 4.47
                                   |S|^2 moves by 1e-2 for a 0.1-cell change of the radius or a 3e-4
                                   change of m, and the scheme's own dispersion at 50 cells per interior
                                   wavelength lowers m by 6.2e-4 (along an axis): against the series at
                                   the lattice's x and m the error is 1.0e-2 instead of 2.5e-2
  sphere eps 2, a/lambda = 1       0.9 / 0.9 / 1.4e-3 at phi 0/45/90
                                   (1.9 / 2.0 / 1.8e-3)
  sphere eps 2, a/lambda = 2       4.6 / 4.6 / 4.8e-3 at phi 0/45/90, 472^3, incident line
                                   (0.18 at every phi); at twice the resolution (944^3)
                                   4.2 / 4.1 / 4.5e-3; backscatter 56-57 against the series' 162
                                   at both resolutions (the paper too reports its largest error there)
  PEC cylinder, a/lambda = 0.1     1.8e-2   (1.5e-2)   min/max 0.411/1.03  (0.428/1.05)
  PEC cylinder, a/lambda = 1       2.7e-3   (3.0e-3)   min/max 1.68/34.2   (1.82/34.2)
  PEC cylinder, a/lambda = 10      3.7e-4   (7.2e-4)   min/max 7.27/2688   (8.81/2.6e3)
The bounds are those values with a margin.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mie

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


# a/lambda = 2 sphere (keyed by lambda_eps/dx): measured 4.6 / 4.6 / 4.8e-3 at
# lambda_eps/dx ~ 50 (the paper: 0.18) and 4.2 / 4.1 / 4.5e-3 at ~100
SPHERE2_BOUND = {50: 6e-3, 100: 5.5e-3}


def nrms(S, ref):
    return float(np.sqrt(np.mean((S - ref) ** 2)) / ref.max())


def lattice_effective(eps_in, lam, a):
    """Size parameter and refractive index the lattice realises at the
    source frequency omega = 2 pi / (3 lambda): the wave numbers of the
    scheme's own dispersion along an axis (oracle.analytic) outside and
    inside the medium, x = k_out a, m = k_in / k_out."""
    from scipy.optimize import brentq

    from oracle import analytic as A

    om = 2 * np.pi / (3 * lam)
    k_out = A.k_vacuum_axis(om)
    g = om * 3 * np.sqrt(eps_in)
    k_in = brentq(lambda k: A.dispersion_axis(k, eps_in) - om, 0.5 * g, min(1.5 * g, 3.0), xtol=1e-15)
    return k_out * a, k_in / k_out


CYLINDERS = [
    # eps, lambda/dx, a/dx, L/a, periods, bound, paper's normalised RMS
    (2.0, 100, 100, 10, 60, 2e-3, 7.8e-4),
    (2.0, 1000, 100, 20, 30, 8e-3, 8.4e-3),
    (2.0, 100, 1000, 4, 100, 5e-3, 1.3e-3),
    (5.0, 112, 112, 10, 150, 3e-3, 1.0e-3),
    (10.0, 158, 158, 10, 150, 5e-3, 2.3e-3),
    (20.0, 224, 224, 10, 150, 3e-2, 6.6e-3),
]


@pytest.mark.parametrize("eps_in,lam,a,L_over_a,periods,bound,paper", CYLINDERS,
                         ids=lambda v: str(v))
def test_cylinder_at_paper_resolution(P, eps_in, lam, a, L_over_a, periods, bound, paper):
    Wl = 32
    n = int(round(L_over_a * a)) + 2 * Wl
    T = int(3 * lam)
    steps = periods * T
    half = np.ceil(a) + max(6, np.ceil(lam / 4)) + 0.5
    case = W.cylinder_case(eps_in, "TM", n=n, a=float(a), lam=float(lam), W=Wl, steps=steps, half=half)
    say("cylinder", eps_in, lam, a, n, steps)
    sims = []
    for c in (W.vacuum_companion(case), case):
        kh, eh = W.plane_wave_2d(0.0, "TM")
        s = P.Simulation(n, n, 1, pol="TM", precision="fp32", absorb=c.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(c.eps)
        s.set_source(c.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.set_ntff(c.box_lo, c.box_hi, *c.window)
        s.step(steps)
        sims.append(s)
    inc, tot = sims
    th = np.arange(0.0, 180.01, 0.5)
    S1 = tot.farfield(th, incident=inc)
    tot.set_ntff(case.box_lo, case.box_hi, steps, T)     # one more period: steady state
    tot.step(T)
    S2 = tot.farfield(th, incident=inc)
    ref = mie.cylinder_S2(th, 2 * np.pi * a / lam, np.sqrt(eps_in), "TM")
    e, drift = nrms(S2, ref), nrms(S2, S1)
    # the same series at the lattice's own x and m (second-order dispersion)
    xe, me = lattice_effective(eps_in, lam, a)
    ref_e = mie.cylinder_S2(th, xe, me, "TM")
    e_eff, e_disp = nrms(S2, ref_e), nrms(ref_e, ref)
    say(f"  nRMS {e:.3e} (paper {paper:.1e}), window drift {drift:.1e}, max {S2.max():.4g} vs {ref.max():.4g}; "
        f"vs the series at the lattice's x, m ({xe:.6f}, {me:.6f}): {e_eff:.3e}; that series vs the nominal one "
        f"{e_disp:.3e}")
    assert drift < 1e-3
    assert e < bound
    if eps_in == 20.0:
        # at m = 4.47 the series moves by 2.3e-2 between the nominal and the
        # lattice's x, m; most of the error is that second-order dispersion
        assert e_eff < 0.6 * e
    for s in sims:
        s.close()


PEC_CYLINDERS = [
    # lambda/dx, a/dx, L/a, periods, bound, paper's normalised RMS
    (500, 50, 20, 20, 2.5e-2, 1.5e-2),
    (50, 50, 10, 60, 4e-3, 3.0e-3),
    (50, 500, 4, 100, 1e-3, 7.2e-4),
]


@pytest.mark.parametrize("lam,a,L_over_a,periods,bound,paper", PEC_CYLINDERS, ids=lambda v: str(v))
def test_pec_cylinder_at_paper_resolution(P, lam, a, L_over_a, periods, bound, paper):
    """Section 3.2.1: PEC cylinders at a / lambda = 0.1, 1, 10 with
    min(a, lambda)/dx = 50 and the paper's L/a, TM; conductor cells read as
    zero-E cells (no rule is printed in the paper)."""
    Wl = 32
    n = int(round(L_over_a * a)) + 2 * Wl
    T = int(3 * lam)
    steps = periods * T
    half = np.ceil(a) + max(6, np.ceil(lam / 4)) + 0.5
    case = W.cylinder_case(1.0, "TM", n=n, a=float(a), lam=float(lam), W=Wl, steps=steps, half=half)
    mask = W.circle(n, float(a), 2.0) > 1.0
    say("pec cylinder", lam, a, n, steps)
    sims = []
    for pec in (False, True):
        kh, eh = W.plane_wave_2d(0.0, "TM")
        s = P.Simulation(n, n, 1, pol="TM", precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        if pec:
            s.set_pec(mask)
        s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
        s.step(steps)
        sims.append(s)
    inc, tot = sims
    th = np.arange(0.0, 180.01, 0.5)
    S1 = tot.farfield(th, incident=inc)
    tot.set_ntff(case.box_lo, case.box_hi, steps, T)     # one more period: steady state
    tot.step(T)
    S2 = tot.farfield(th, incident=inc)
    ref = mie.cylinder_S2(th, 2 * np.pi * a / lam, None, "TM")
    aeq = np.sqrt(np.count_nonzero(mask) / np.pi)
    e, drift = nrms(S2, ref), nrms(S2, S1)
    e_in = min(nrms(S2, mie.cylinder_S2(th, 2 * np.pi * (a - d) / lam, None, "TM")) for d in (0.25, 0.5))
    say(f"  nRMS {e:.3e} (paper {paper:.1e}; series at a - 1/4..1/2 cell: {e_in:.3e}; area-equivalent "
        f"radius {aeq:.3f}), window drift {drift:.1e}, min/max {S2.min():.4g}/{S2.max():.4g} vs "
        f"{ref.min():.4g}/{ref.max():.4g}")
    assert drift < 1e-3
    assert e < bound
    for s in sims:
        s.close()


def test_sphere_at_paper_resolution(P):
    """Sphere eps 2, a/lambda = 1, a/dx = 71 (lambda_eps/dx = 50), L/a = 4."""
    lam = a = 71.0
    Wl = 24
    n = 4 * 71 + 2 * Wl
    T = int(3 * lam)
    steps = 40 * T
    case = W.sphere_case(n=n, x_size=2 * np.pi * a / lam, lam=lam, eps_in=2.0, W=Wl, steps=steps,
                         half=np.ceil(a) + 18 + 0.5)
    say("sphere", n, steps)
    sims = []
    for e in (None, case.eps):
        s = P.Simulation(n, n, n, pol="3D", precision="fp32", absorb=(Wl,) * 3, sigma_max=W.SIGMA_MAX)
        if e is not None:
            s.set_permittivity(e)
        s.set_source(lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
        s.step(steps)
        sims.append(s)
    inc, tot = sims
    th = np.arange(0.0, 180.01, 0.5)
    first = {ph: tot.farfield(th, np.full_like(th, ph), incident=inc) for ph in (0.0, 45.0, 90.0)}
    tot.set_ntff(case.box_lo, case.box_hi, steps, T)
    tot.step(T)
    for ph, paper in ((0.0, 1.9e-3), (45.0, 2.0e-3), (90.0, 1.8e-3)):
        S = tot.farfield(th, np.full_like(th, ph), incident=inc)
        ref = mie.sphere_S2(th, ph, 2 * np.pi, np.sqrt(2.0))
        e, drift = nrms(S, ref), nrms(S, first[ph])
        say(f"  phi {ph}: nRMS {e:.3e} (paper {paper:.1e}), drift {drift:.1e}")
        assert drift < 1e-3
        assert e < 3e-3
    for s in sims:
        s.close()


def _sphere_with_line(P, lam, a, Wl, periods):
    """Sphere eps 2 of radius a at wavelength lam (cells), L/a = 3 (Table
    dielectric_sphere_er_2) plus a layer of Wl cells; the exact incident line
    replaces the companion run (a companion of the larger grid would not
    fit next to it).  Returns |S|^2 at phi = 0/45/90 over 0..180 degrees of
    the last window and the drift to the window one period earlier."""
    n = int(round(3 * a)) + 2 * Wl
    T = int(round(3 * lam))
    steps = periods * T
    case = W.sphere_case(n=n, x_size=2 * np.pi * a / lam, lam=lam, eps_in=2.0, W=Wl, steps=steps,
                         half=np.ceil(a) + 18 + 0.5)
    say("sphere a/lambda = 2", n, lam, a, steps)
    s = P.Simulation(n, n, n, pol="3D", precision="fp32", absorb=(Wl,) * 3, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    case.eps = None
    s.set_source(lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
    s.set_ntff(case.box_lo, case.box_hi, *case.window)
    s.set_incident_line(True)
    done = 0
    while done < steps:             # progress lines for long runs
        k = min(1024, steps - done)
        s.step(k)
        done += k
        if n > 600:
            import torch

            torch.cuda.synchronize()
            say(f"  step {done} / {steps}")
    th = np.arange(0.0, 180.01, 0.5)
    first = {ph: s.farfield(th, np.full_like(th, ph)) for ph in (0.0, 45.0, 90.0)}
    s.set_ntff(case.box_lo, case.box_hi, steps, T)
    s.step(T)
    out = {}
    for ph in (0.0, 45.0, 90.0):
        S = s.farfield(th, np.full_like(th, ph))
        ref = mie.sphere_S2(th, ph, 2 * np.pi * a / lam, np.sqrt(2.0))
        out[ph] = (nrms(S, ref), nrms(S, first[ph]), S, ref)
    s.close()
    return out


def test_sphere_a_over_lambda_2_at_paper_resolution(P):
    """Sphere eps 2, a/lambda = 2 at the paper's lambda_eps/dx ~ 50 (a/dx =
    141, L/a = 3; 472^3 with the layer).  The paper reports a normalised RMS
    of 0.18 at every phi here and names a finer grid as future work."""
    lam = 212.0 / 3.0                  # 3 lambda integral; lambda_eps = 49.97 cells
    res = _sphere_with_line(P, lam, 2 * lam, 24, 26)
    for ph, (e, drift, S, ref) in res.items():
        say(f"  phi {ph}: nRMS {e:.3e} (paper 0.18), drift {drift:.1e}, back {S[-1]:.4g} vs {ref[-1]:.4g}")
        assert drift < 1e-3
        assert e < SPHERE2_BOUND[50]


@pytest.mark.skipif(not os.environ.get("LBM_EM_LONG_TESTS"),
                    reason="944^3 run of about 5 minutes; set LBM_EM_LONG_TESTS=1")
def test_sphere_a_over_lambda_2_at_double_resolution(P):
    """The same sphere at lambda_eps/dx ~ 100 (a/dx = 283; 944^3 with a
    48-cell layer, 185 GB of FP32 state), the resolution the paper names as
    future work in section 3.4."""
    lam = 424.0 / 3.0
    res = _sphere_with_line(P, lam, 2 * lam, 48, 26)
    for ph, (e, drift, S, ref) in res.items():
        say(f"  phi {ph}: nRMS {e:.3e} (paper at half this resolution 0.18), drift {drift:.1e}, "
            f"back {S[-1]:.4g} vs {ref[-1]:.4g}")
        assert drift < 1e-3
        assert e < SPHERE2_BOUND[100]
