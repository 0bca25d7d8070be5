"""Full-length parity against stored oracle results.

The workloads at their full sizes and step counts, in the launch
configuration the benchmark times, against FP64 oracle runs written by
tests/golden/make_golden.py (which calls only oracle/ and workloads/):

* the 2-D circular cylinder, 1024^2, a = 25.5, lambda = 32, W = 32, 8000
  steps (DFT over steps 7904..7999), eps_r in {1.5, 2.25, 4.0}, TM and TE,
  with the eps_r = 1 companion runs: contour phasors element by element,
  |S(theta)|^2 at 720 angles angle by angle, and the step-8000 fields on
  ten rows and ten columns through the layers, the contour and the
  scatterer;
* two instances of the seeded 64-instance batch (a hexagon at 10.9 degrees,
  a circle at 53.9 degrees; 6000 steps) stepped inside the full batch.

Bars: FP32 <= 1e-4 relative L2 on fields, <= 1e-3 on |S|^2 (see
paritycheck); FP64 <= 1e-12 on fields and 1e-11 on phasors.
"""
import os

import numpy as np
import pytest

import workloads as W
from paritycheck import assert_intensity, max_rel, rel_l2, say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_11042_amd as P

    return P


def _load(name):
    return np.load(os.path.join(HERE, "golden", name))


def _lines(E, H, lines, comps):
    F = np.concatenate([E[0], H[0]], axis=-1)[..., list(comps)].astype(np.float64)
    rows = np.stack([F[l, :, :] for l in lines])
    cols = np.stack([F[:, l, :] for l in lines])
    return np.stack([rows, cols], axis=1)


def _comps(pol):
    return (2, 3, 4) if pol == "TM" else (0, 1, 5)


@pytest.fixture(scope="module", params=["fp32", "fp64"])
def cylinder_job(P, request):
    """The benchmark's eight solves (its autotuned launch shapes), 8000 steps."""
    import bench

    prec = request.param
    say("cylinder job", prec)
    sims = bench.cylinder_workload(P.Simulation, W, 8000, precision=prec)
    for pol, eps_in, s in sims:
        s.step(8000)
        assert s.t == 8000
    yield prec, sims
    for _, _, s in sims:
        s.close()


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_cylinder_full_length_vs_oracle(cylinder_job, pol):
    prec, sims = cylinder_job
    g = _load("cylinder1024_8000.npz")
    theta = g["theta_rel_deg"]
    lines = tuple(int(v) for v in g["lines"])
    inc = [s for p, e, s in sims if p == pol and e == 1.0][0]
    ptol = 1e-11 if prec == "fp64" else 1e-4
    for eps_in in (1.0, 1.5, 2.25, 4.0):
        s = [s for p, e, s in sims if p == pol and e == eps_in][0]
        tag = f"{pol}_vac" if eps_in == 1.0 else f"{pol}_eps{eps_in:g}"
        say(prec, tag, "tile", s.get_fusion(), s.get_fusion_tile())
        X, probe = s.phasors()
        Xo, po = g[f"{tag}_phasors"], g[f"{tag}_probe"]
        perr = max_rel(X, Xo)
        say(prec, tag, "phasors max err / max", perr, "probe", abs(probe - po).max() / abs(Xo).max())
        assert perr <= ptol and np.abs(probe - po).max() <= ptol * np.abs(Xo).max()
        if f"{tag}_fields" in g:
            E, H = s.fields()
            Fg, Fo = _lines(E, H, lines, _comps(pol)), g[f"{tag}_fields"]
            if prec == "fp64":
                err = max_rel(Fg, Fo)
                say(prec, tag, "fields max err / max", err)
                assert err <= 1e-12
            else:
                err = rel_l2(Fg, Fo)
                say(prec, tag, "fields rel L2", err)
                assert err <= 1e-4
                # and line by line: every stored row and column on its own
                for i in range(len(lines)):
                    for k in range(2):
                        if np.any(Fo[i, k]):
                            assert rel_l2(Fg[i, k], Fo[i, k]) <= 1e-4, (tag, lines[i], k)
        if eps_in != 1.0:
            S = s.farfield(theta, incident=inc)
            assert_intensity(S, g[f"{tag}_S2"], 1e-10 if prec == "fp64" else 1e-3, f"{prec} {tag}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_instances_full_length_vs_oracle(P, prec):
    """The seeded 64-instance batch (sides 256..448, 6000 steps) in one
    Batch; instances 1 (hexagon, 10.9 deg) and 2 (circle, 53.9 deg) and
    their companions against the oracle."""
    g = _load("batch_instances_6000.npz")
    cases = W.batch_cases(64)
    ids = [int(i) for i in g["ids"]]
    sims = []
    for c in cases + [W.vacuum_companion(cases[i]) for i in ids]:
        kh, eh = W.plane_wave_2d(c.theta_deg, c.pol)
        s = P.Simulation(c.nx, c.ny, 1, pol=c.pol, precision=prec, absorb=c.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(c.eps)
        s.set_source(c.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.set_ntff(c.box_lo, c.box_hi, *c.window)
        sims.append(s)
    b = P.Batch(sims)
    say("batch", prec, "groups", b.groups)
    b.step(6000)
    theta = g["theta_rel_deg"]
    for j, i in enumerate(ids):
        c = cases[i]
        lines = tuple(int(v) for v in g[f"b{i}_lines"])
        for tag, s in ((f"b{i}", sims[i]), (f"b{i}_vac", sims[64 + j])):
            assert s.t == 6000
            X, probe = s.phasors()
            perr = max_rel(X, g[f"{tag}_phasors"])
            E, H = s.fields()
            Fg, Fo = _lines(E, H, lines, _comps(c.pol)), g[f"{tag}_fields"]
            ferr = max_rel(Fg, Fo) if prec == "fp64" else rel_l2(Fg, Fo)
            say(prec, tag, c.shape, c.nx, "phasor err", perr, "field err", ferr)
            assert perr <= (1e-11 if prec == "fp64" else 1e-4)
            assert ferr <= (1e-12 if prec == "fp64" else 1e-4)
        S = sims[i].farfield(theta, incident=sims[64 + j])     # angles from the incidence direction
        assert_intensity(S, g[f"b{i}_S2"], 1e-10 if prec == "fp64" else 1e-3, f"{prec} batch {i}")
    b.close()
    for s in sims:
        s.close()
