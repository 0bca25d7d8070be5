"""Full-size workloads on the GPU against the physics the paper checks:
Fresnel at a planar interface (section 3.1), Lorenz-Mie for the circular
cylinder (section 3.2) and the sphere (section 3.4).

At these sizes the FP64 oracle needs minutes per run, so the checks are
properties that hold at any size (mirror symmetry of normal incidence) and
agreement with the analytic references at the accuracy the resolution
allows (normalised RMS of Eq. rms_error).  The bounds are the measured
values of this implementation with a margin, far below what a wrong
coupling, source or transform would give; the series are evaluated at the
staircase's area-equivalent radius, which is what a cell-centre staircase
resolves at these grids (radius 25.5 cells, interior wavelength down to 16
cells).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mie
from oracle.analytic import fresnel_normal, fresnel_oblique

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


def nrms(S, ref):
    return float(np.sqrt(np.mean((S - ref) ** 2)) / ref.max())


def _run2d(P, case, prec="fp32"):
    kh, eh = W.plane_wave_2d(case.theta_deg, case.pol)
    s = P.Simulation(case.nx, case.ny, 1, pol=case.pol, precision=prec, absorb=case.absorb,
                     sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
    if case.box_lo is not None:
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
    s.step(case.steps)
    return s


# normalised RMS bounds vs Mie at the area-equivalent radius: measured
# 0.18 / 1.09 / 0.76 % (TM eps 1.5 / 2.25 / 4), 0.11 / 0.89 / 0.70 % (TE eps 1.5 /
# 2.25 / 4); 2 % leaves room for rounding and stays well below what a wrong
# coupling, source or transform gives (tens of per cent)
CYL_BOUND = 0.02


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_cylinder_1024_vs_mie(P, pol):
    """1024^2, a = 25.5 (x = 5.007), lambda = 32, W = 32, 8000 steps, FP32;
    |S(theta)|^2 at 0.5 degrees over the full circle."""
    th = np.arange(0.0, 360.0, 0.5)
    inc = _run2d(P, W.vacuum_companion(W.cylinder_case(1.0, pol, n=1024)))
    for eps_in in (1.5, 2.25, 4.0):
        case = W.cylinder_case(eps_in, pol, n=1024)
        s = _run2d(P, case)
        S = s.farfield(th, incident=inc)
        aeq = np.sqrt(np.count_nonzero(case.eps > 1) / np.pi)
        k = 2 * np.pi / case.lam
        ref = mie.cylinder_S2(th, k * aeq, np.sqrt(eps_in), pol)
        ref_nom = mie.cylinder_S2(th, k * case.radius, np.sqrt(eps_in), pol)
        e, e_nom = nrms(S, ref), nrms(S, ref_nom)
        sym = np.abs(S[1:360] - S[719:360:-1]).max() / S.max()
        say(pol, eps_in, "nRMS vs Mie(a_eq)", e, "vs Mie(a)", e_nom, "max S", S.max(), ref.max(),
            "mirror asym", sym)
        assert sym < 1e-4
        assert e < CYL_BOUND
        s.close()


@pytest.mark.parametrize("n", [384, 512])
def test_sphere_vs_mie(P, n):
    """384^3 and 512^3 sphere, x = 6 at lambda = 24, eps 2.25, W = 24, 4000
    steps, FP32, k along +z, E along +x; |S(theta, phi)|^2 in the planes
    phi = 0, 45, 90."""
    case = W.sphere_case(n=n)
    say("sphere", n)
    sims = []
    for e in (np.ones(1), case.eps):
        s = P.Simulation(n, n, n, pol="3D", precision="fp32", absorb=(case.W,) * 3,
                         sigma_max=W.SIGMA_MAX)
        if e.size > 1:
            s.set_permittivity(e)
        s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
        s.step(case.steps)
        sims.append(s)
    inc, tot = sims
    th = np.arange(0.0, 180.01, 0.5)
    aeq = (np.count_nonzero(case.eps > 1) * 3 / (4 * np.pi)) ** (1 / 3)
    k = 2 * np.pi / case.lam
    for phi in (0.0, 45.0, 90.0):
        S = tot.farfield(th, np.full_like(th, phi), incident=inc)
        ref = mie.sphere_S2(th, phi, k * aeq, 1.5)
        e = nrms(S, ref)
        say("sphere phi", phi, "nRMS vs Mie(a_eq)", e, "max", S.max(), ref.max(), "a_eq", aeq)
        assert e < 0.02     # measured 1.1-1.2 % at lambda_eps = 16 cells (384^3)
    for s in sims:
        s.close()


@pytest.mark.parametrize("theta,pol", [(0.0, "TM"), (30.0, "TM"), (0.0, "TE"), (30.0, "TE")])
def test_fresnel_256x128(P, theta, pol):
    """Planar interface 256 x 128, eps 2.25 for x >= 128, W = 20, 3000 steps:
    reflected / transmitted amplitudes from the fields of the last period
    against Fresnel (the oracle test's reading and bounds)."""
    case = W.fresnel_case(theta, pol, ny=128)
    T = W.period_steps(case.lam)
    amps = []
    for c in (case, W.vacuum_companion(case)):
        kh, eh = W.plane_wave_2d(theta, pol)
        s = P.Simulation(c.nx, c.ny, 1, pol=pol, precision="fp32", absorb=c.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(c.eps)
        s.set_source(c.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.step(c.steps - T)
        acc = np.zeros((case.nx, 3), complex)
        omega = 2 * np.pi / (3 * c.lam)
        for t in range(c.steps - T, c.steps):      # DFT of row y = 0 over the last period
            E, _ = s.fields()
            acc += (2.0 / T) * E[0, 0] * np.exp(-1j * omega * t)
            s.step(1)
        amps.append(acc)
    tot, inc = amps
    amp = lambda v: np.sqrt(np.sum(np.abs(v) ** 2, axis=1))
    vac, die = slice(24, 124), slice(132, 232)
    r = np.mean(amp(tot[vac] - inc[vac]) / amp(inc[vac]))
    t = np.mean(amp(tot[die]) / amp(inc[die]))
    if theta == 0:
        r_ref, t_ref = fresnel_normal(2.25)
    else:
        r_ref, t_ref, _ = fresnel_oblique(2.25, theta, "s" if pol == "TM" else "p")
    say("fresnel", theta, pol, "r", r, abs(r_ref), "t", t, abs(t_ref))
    assert abs(r - abs(r_ref)) < (0.01 if theta == 0 else 0.03)
    assert abs(t - abs(t_ref)) < 0.01


SWEEP = [(1.5, 1.0), (4.0, 1.0), (20.0, 1.0), (80.0, 1.0), (200.0, 1.0),
         (1.0, 1.5), (1.0, 4.0), (1.0, 20.0), (1.0, 80.0), (1.0, 200.0)]


def _row_dft_device(P, case, pol, mu=None):
    """E phasor of the single-row grid over the last period (DFT of the
    library's fields on the device)."""
    import torch

    kh, eh = W.plane_wave_2d(0.0, pol)
    s = P.Simulation(case.nx, 1, 1, pol=pol, precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    if mu is not None:
        s.set_permeability(mu)
    s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
    w0, T = case.window
    s.step(w0)
    c = 2 if pol == "TM" else 1
    omega = 2 * np.pi / (3 * case.lam)
    acc = torch.zeros(case.nx, dtype=torch.complex128, device="cuda")
    for t in range(w0, w0 + T):
        E, _ = s.fields_device()
        acc += E[0, 0, :, c].double() * complex(np.exp(-1j * omega * t) * 2.0 / T)
        s.step(1)
    out = acc.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_material_sweep_section_3_1(P, pol):
    """Section 3.1's sweep on the GPU: normal incidence onto a half space
    with eps_r from 1.5 to 200 (mu_r = 1) and mu_r from 1.5 to 200 (eps_r =
    1), 20 cells per wavelength inside the medium, against Eq. ref_trans.
    Bounds as the oracle's sweep test: reflection within 0.005, transmission
    within 2 % (measured about 1 %: the scheme's second-order error at 20
    cells per inner wavelength)."""
    companions = {}
    for eps_in, mu_in in SWEEP:
        case = W.planar_sweep_case(eps_in, mu_in, pol=pol)
        key = (case.nx, case.lam)
        if key not in companions:
            companions[key] = _row_dft_device(P, W.vacuum_companion(case), pol)
        inc = companions[key]
        tot = _row_dft_device(P, case, pol, case.extra["mu"] if mu_in != 1.0 else None)
        x0 = case.extra["x0"]
        vac = slice(20 + 8, x0 - 8)
        die = slice(x0 + 8, case.nx - 20 - 8)
        r = np.abs(tot[vac] - inc[vac]) / np.abs(inc[vac])
        t = np.abs(tot[die]) / np.abs(inc[die])
        r_ref, t_ref = fresnel_normal(eps_in, mu_in)
        say("sweep", pol, eps_in, mu_in, "r", r.mean(), abs(r_ref), "t", t.mean(), t_ref)
        assert r.std() < 0.002 and t.std() < 0.01 * t_ref, (r.std(), t.std())
        assert abs(r.mean() - abs(r_ref)) < 0.005, (eps_in, mu_in, r.mean(), r_ref)
        assert abs(t.mean() / t_ref - 1.0) < 0.02, (eps_in, mu_in, t.mean(), t_ref)
