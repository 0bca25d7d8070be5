"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Bars: FP64 library build vs oracle <= 1e-12 (relative to the field scale);
FP32 library vs oracle <= 1e-4 relative L2 on field snapshots and <= 1e-3
normalised on |S|^2 (angular intensity).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ntff, run
from oracle.core import Oracle
from paritycheck import assert_intensity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11042_amd import Simulation

    return Simulation


def rel_l2(a, b):
    return float(np.sqrt(np.sum((np.asarray(a, float) - b) ** 2) / np.sum(b ** 2)))


def make_pair(Sim, nx, ny, nz, pol, prec, absorb, eps, lam, khat, ehat, ramp=3.0):
    s = Sim(nx, ny, nz, pol=pol, precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(eps)
    s.set_source(lam, khat, ehat, 1.0, ramp)
    o = Oracle(nx, ny, nz, absorb, W.SIGMA_MAX)
    o.set_eps(eps)
    center = [(m - 1) / 2.0 for m in (nx, ny, nz)]
    if nz == 1:
        center[2] = 0.0
    o.set_source(lam, khat, ehat, 1.0, ramp, center)
    return s, o


def compare_fields(s, o, prec, tag):
    Eg, Hg = s.fields()
    Eo, Ho = o.fields()
    scale = max(np.abs(Eo).max(), np.abs(Ho).max())
    if scale == 0.0:   # source ramp still at zero: both must be exactly zero
        assert not np.any(Eg) and not np.any(Hg), tag
        return
    assert scale > 1e-3 or o.t < 20, "the wave has not entered the domain"
    if prec == "fp64":
        err = max(np.abs(Eg - Eo).max(), np.abs(Hg - Ho).max()) / scale
        say(tag, "fp64 max rel err", err)
        assert err <= 1e-12, (tag, err)
    else:
        err = rel_l2(np.concatenate([Eg.ravel(), Hg.ravel()]), np.concatenate([Eo.ravel(), Ho.ravel()]))
        say(tag, "fp32 rel L2", err)
        assert err <= 1e-4, (tag, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("theta,pol", [(0.0, "TM"), (30.0, "TM"), (0.0, "TE"), (30.0, "TE")])
def test_fresnel_config_fields(gpu, prec, theta, pol):
    """Planar interface, 256 x 128, eps 2.25 half space, W = 20, lambda = 32,
    3000 steps (the small configuration at full size)."""
    case = W.fresnel_case(theta, pol, ny=128)
    say("fresnel", prec, theta, pol)
    kh, eh = W.plane_wave_2d(theta, pol)
    s, o = make_pair(gpu, case.nx, case.ny, 1, pol, prec, case.absorb, case.eps, case.lam, kh, eh)
    s.step(case.steps)
    o.step(case.steps)
    assert s.t == o.t == case.steps
    compare_fields(s, o, prec, f"fresnel {pol} {theta}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_grid_mixed_boundaries(gpu, prec):
    """Sizes that leave ragged tiles (67 x 45), x periodic / y absorbing,
    random dielectric blobs, oblique TE source."""
    nx, ny = 67, 45
    rng = np.random.default_rng(11)
    eps = 1.0 + (rng.random((1, ny, nx)) < 0.15) * rng.uniform(0.5, 3.0, (1, ny, nx))
    eps[:, :10, :] = 1.0
    eps[:, -10:, :] = 1.0
    th = np.deg2rad(70.0)
    kh = [np.cos(th), np.sin(th), 0.0]
    eh = [-np.sin(th), np.cos(th), 0.0]
    say("ragged", prec)
    s, o = make_pair(gpu, nx, ny, 1, "TE", prec, (0, 9, 0), eps, 10.0, kh, eh, ramp=1.0)
    for n in (1, 7, 130):     # mixes eager steps and graph chunks
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"ragged t={o.t}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_three_d_sphere_fields(gpu, prec):
    n = 40
    case = W.sphere_case(n=n, x_size=3.0, lam=10.0, eps_in=2.25, W=8, steps=260, half=9.5)
    say("3d", prec)
    s, o = make_pair(gpu, n, n, n, "3D", prec, (8, 8, 8), case.eps, case.lam, [0, 0, 1.0], [1.0, 0, 0],
                     ramp=1.0)
    s.step(case.steps)
    o.step(case.steps)
    compare_fields(s, o, prec, "3d sphere")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_source_phase_tables(gpu, prec):
    """The incident wave comes from per-axis phase tables: oblique incidence
    with all three axis phases non-zero (3-D), and a ramp of 1.5 periods
    (an odd number of table entries before the per-axis tables), checked
    during and after the ramp."""
    th = np.deg2rad(35.0)
    kh = [np.cos(th), np.sin(th), 0.0]
    eps = np.ones((1, 50, 70))
    eps[:, 20:30, 30:42] = 2.5
    s, o = make_pair(gpu, 70, 50, 1, "TM", prec, (12, 12, 0), eps, 10.0, kh, [0, 0, 1.0], ramp=1.5)
    for n in (20, 25, 105):
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"tables 2-D t={o.t}")
    k3 = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    e3 = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    eps3 = np.ones((24, 24, 24))
    eps3[9:15, 9:15, 9:15] = 2.0
    s, o = make_pair(gpu, 24, 24, 24, "3D", prec, (6, 6, 6), eps3, 10.0, list(k3), list(e3), ramp=1.5)
    for n in (30, 60):
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"tables 3-D t={o.t}")


X3_TILES = {"fp32": [(64, 16), (64, 8), (32, 16), (128, 8), (256, 4), (128, 4)],
            "fp64": [(32, 16), (32, 8), (16, 16), (64, 8), (128, 4)]}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_three_d_two_steps_per_launch_is_bit_identical(gpu, prec):
    """The 3-D z march with two steps per launch reproduces one step per
    launch bit for bit (fields and DFT phasors) for every 3-D tile, on a
    ragged grid with one periodic axis (x or y), odd step counts, and z
    chunks that do not divide the grid."""
    nx, ny, nz = 70, 37, 29
    rng = np.random.default_rng(9)
    eps = np.ones((nz, ny, nx))
    eps[9:20, 12:25, 25:45] = 1.0 + rng.uniform(0.5, 2.0, (11, 13, 20))
    k3 = np.array([1.0, 0.4, 0.7]) / np.linalg.norm([1.0, 0.4, 0.7])
    e3 = np.cross(k3, [0.0, 0.0, 1.0])
    e3 /= np.linalg.norm(e3)
    for absorb in ((10, 0, 6), (0, 8, 6)):
        runs = []
        for fuse, tile in [(1, (0, 0))] + [(2, t) for t in X3_TILES[prec]]:
            s = gpu(nx, ny, nz, pol="3D", precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
            s.set_permittivity(eps)
            s.set_source(10.0, list(k3), list(e3), 1.0, 1.0)
            s.set_ntff((20, 9, 8), (50, 28, 21), 100, 30)
            s.set_fusion(fuse, tile)
            for n in (3, 131, 1):
                s.step(n)
            runs.append((s.fields(), s.phasors()))
            say("3-D fusion", prec, absorb, fuse, tile, s.t)
            s.close()
        (E1, H1), (X1, p1) = runs[0]
        assert np.abs(E1).max() > 0
        for (E2, H2), (X2, p2) in runs[1:]:
            assert np.array_equal(E1, E2) and np.array_equal(H1, H2)
            assert np.array_equal(X1, X2) and np.array_equal(p1, p2)


def test_graph_replay_equals_eager(gpu):
    """step(n) replays captured graphs in 64-step chunks; results must be
    bit-identical to single eager steps."""
    case = W.cylinder_case(2.25, "TM", n=128, a=10.0, lam=16.0, W=16, steps=200, half=14.5)
    kh, eh = W.plane_wave_2d(0.0, "TM")
    sims = []
    for _ in range(2):
        s = gpu(128, 128, 1, pol="TM", precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(case.eps)
        s.set_source(case.lam, kh, eh)
        sims.append(s)
    say("graph vs eager")
    sims[0].step(200)
    for _ in range(200):
        sims[1].step(1)
    E0, H0 = sims[0].fields()
    E1, H1 = sims[1].fields()
    assert np.array_equal(E0, E1) and np.array_equal(H0, H1)


def _gpu_case(Sim, case, prec):
    kh, eh = W.plane_wave_2d(case.theta_deg, case.pol)
    s = Sim(case.nx, case.ny, 1, pol=case.pol, precision=prec, absorb=case.absorb, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
    w0, wl = case.window
    s.set_ntff(case.box_lo, case.box_hi, w0, wl)
    s.step(case.steps)
    return s


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_cylinder_pipeline_phasors_and_intensity(gpu, pol):
    """Whole path on a small cylinder (192^2, a = 10.5, lambda = 32, 2400
    steps): contour DFT phasors and |S(theta)|^2 at 0.5 degree resolution
    against the oracle's DFT + NTFF."""
    case = W.cylinder_case(2.25, pol, n=192, a=10.5, lam=32.0, W=32, steps=2400, half=19.5)
    inc_case = W.vacuum_companion(case)
    say("pipeline", pol)
    tot_o = run.run_2d(case, W.SIGMA_MAX, W.RAMP_PERIODS)
    inc_o = run.run_2d(inc_case, W.SIGMA_MAX, W.RAMP_PERIODS)
    th = np.arange(0, 360, 0.5)
    S_o = run.intensity_2d(case, tot_o, inc_o, th)
    for prec, ptol, stol in (("fp64", 1e-11, 1e-10), ("fp32", 1e-4, 1e-3)):
        tot_g = _gpu_case(gpu, case, prec)
        inc_g = _gpu_case(gpu, inc_case, prec)
        X, probe = tot_g.phasors()
        scale = np.abs(tot_o["phasors"]).max()
        perr = np.abs(X - tot_o["phasors"]).max() / scale
        say(pol, prec, "phasor err", perr)
        assert perr <= ptol
        assert np.abs(probe - tot_o["probe"]).max() <= ptol * scale
        S_g = tot_g.farfield(th, incident=inc_g)
        assert_intensity(S_g, S_o, stol, f"pipeline {pol} {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_three_d_pipeline_intensity(gpu, prec):
    """3-D DFT + NTFF on a small sphere (48^3) against the oracle, in the
    two scattering planes phi = 0, 90 degrees and phi = 45."""
    n = 48
    case = W.sphere_case(n=n, x_size=2.5, lam=12.0, eps_in=2.25, W=8, steps=360, half=8.5)
    vac = W.sphere_case(n=n, x_size=2.5, lam=12.0, eps_in=1.0, W=8, steps=360, half=8.5)
    say("3d pipeline", prec)
    tot_o = run.run_3d(case, W.SIGMA_MAX, 1.0)
    inc_o = run.run_3d(vac, W.SIGMA_MAX, 1.0)
    th = np.arange(0, 180.01, 0.5)
    sims = []
    for c in (case, vac):
        s = gpu(n, n, n, pol="3D", precision=prec, absorb=(8, 8, 8), sigma_max=W.SIGMA_MAX)
        s.set_permittivity(c.eps)
        s.set_source(c.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, 1.0)
        s.set_ntff(c.box_lo, c.box_hi, *c.window)
        s.step(c.steps)
        sims.append(s)
    for phi in (0.0, 45.0, 90.0):
        S_o = run.intensity_3d(case, tot_o, inc_o, th, np.full_like(th, phi))
        S_g = sims[0].farfield(th, np.full_like(th, phi), incident=sims[1])
        assert_intensity(S_g, S_o, 1e-10 if prec == "fp64" else 1e-3, f"3d phi {phi} {prec}")


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_full_size_cylinder_grid_short_run(gpu, pol):
    """The 1024^2 cylinder configuration in the launch configuration the
    benchmark times, for 300 steps (the oracle's full-length run takes
    minutes): every tile, the layers and the source against the oracle."""
    case = W.cylinder_case(2.25, pol, n=1024, steps=300)
    kh, eh = W.plane_wave_2d(0.0, pol)
    say("full size short", pol)
    o = Oracle(1024, 1024, 1, case.absorb, W.SIGMA_MAX)
    o.set_eps(case.eps)
    o.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS, [511.5, 511.5, 0.0])
    o.step(case.steps)
    for prec in ("fp32", "fp64"):
        s = gpu(1024, 1024, 1, pol=pol, precision=prec, absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(case.eps)
        s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.step(case.steps)
        compare_fields(s, o, prec, f"1024^2 {pol}")
        s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_every_tile_gives_identical_results(gpu, dim):
    """The tile (cells per thread, block shape) changes speed only: each
    cell's update is independent of it, so results are bit-identical."""
    if dim == 2:
        n = (83, 70, 1)
        case = W.cylinder_case(2.25, "TE", n=83, a=9.0, lam=12.0, W=10, steps=150, half=13.0)
        eps, pol, absorb = case.eps[:, :70, :], "TE", (10, 10, 0)
        kh, eh = W.plane_wave_2d(20.0, "TE")
        tiles = [(1, 64, 4), (2, 64, 4), (4, 64, 4), (4, 256, 1), (2, 32, 8), (4, 16, 16), (1, 128, 1)]
    else:
        n = (36, 30, 28)
        eps = W.sphere_case(n=36, x_size=2.0, lam=9.0, eps_in=2.25, W=6, steps=90, half=8.5).eps[:28, :30, :]
        pol, absorb = "3D", (6, 6, 6)
        kh, eh = [0, 0, 1.0], [1.0, 0, 0]
        tiles = [(1, 64, 4), (2, 64, 4), (4, 64, 4), (4, 32, 2), (2, 256, 1)]
    ref = None
    for prec in ("fp32", "fp64"):
        ref = None
        for vx, bx, by in tiles:
            if prec == "fp64" and vx == 4:
                continue
            say("tile", dim, prec, vx, bx, by)
            s = gpu(*n, pol=pol, precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
            s.set_permittivity(eps)
            s.set_source(9.0 if dim == 3 else 12.0, kh, eh, 1.0, 1.0)
            s.set_tile(vx, bx, by)
            assert s.get_tile() == (vx, bx, by)
            s.step(90 if dim == 3 else 150)
            E, H = s.fields()
            if ref is None:
                ref = (E, H)
            else:
                assert np.array_equal(E, ref[0]) and np.array_equal(H, ref[1]), (vx, bx, by)
            s.close()


def test_autotune_verifies_and_does_not_advance(gpu):
    from paper_2510_11042_amd import LbmEmError

    case = W.cylinder_case(2.25, "TM", n=256, a=12.0, lam=16.0, W=16, steps=120, half=18.5)
    kh, eh = W.plane_wave_2d(0.0, "TM")
    sims = []
    for tune in (False, True):
        s = gpu(256, 256, 1, pol="TM", precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(case.eps)
        s.set_source(case.lam, kh, eh)
        s.step(60)
        if tune:
            rec = s.autotune(launches=5)
            say("autotune", rec)
            assert s.t == 60
        s.step(60)
        sims.append(s)
    assert np.array_equal(sims[0].fields()[0], sims[1].fields()[0])
    with pytest.raises(LbmEmError):
        sims[0].set_tile(3, 64, 4)
    with pytest.raises(LbmEmError):
        sims[0].set_tile(1, 100, 1)


X2_TILES = {"fp32": [(64, 16), (128, 8), (128, 16), (256, 8), (256, 16), (128, 32)],
            "fp64": [(32, 16), (64, 8), (64, 16), (128, 8), (128, 16), (64, 32)]}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_two_steps_per_launch_is_bit_identical(gpu, prec, pol):
    """Temporal blocking (two steps per launch through LDS) reproduces one
    step per launch bit for bit: fields and DFT phasors, for every two-step
    tile, on a ragged grid with one periodic and one absorbing axis (both
    ways round, so ragged tiles meet both the wrap and the clamp), odd step
    counts (graph chunks + fused pairs + a single trailing step), and on a
    1-row grid and a periodic grid smaller than one segment."""
    nx, ny = 203, 77
    rng = np.random.default_rng(5)
    eps = 1.0 + (rng.random((1, ny, nx)) < 0.2) * rng.uniform(0.2, 3.0, (1, ny, nx))
    eps[:, :, :12] = 1.0
    eps[:, :, -12:] = 1.0
    eps[:, :10, :] = 1.0
    eps[:, -10:, :] = 1.0
    th = np.deg2rad(25.0)
    kh = [np.cos(th), np.sin(th), 0.0]
    eh = [0, 0, 1.0] if pol == "TM" else [-np.sin(th), np.cos(th), 0.0]
    tiles = X2_TILES[prec]
    for absorb in ((11, 0, 0), (0, 9, 0)):
        runs = []
        for fuse, tile in [(1, (0, 0))] + [(2, t) for t in tiles]:
            s = gpu(nx, ny, 1, pol=pol, precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
            s.set_permittivity(eps)
            s.set_source(10.0, kh, eh, 1.0, 1.0)
            s.set_ntff((60, 20, 0), (140, 56, 0), 100, 30)
            s.set_fusion(fuse, tile)
            assert s.get_fusion() == fuse
            for n in (3, 131, 1):
                s.step(n)
            runs.append((s.fields(), s.phasors()))
            say("fusion", prec, pol, absorb, fuse, tile, s.t)
            s.close()
        (E1, H1), (X1, p1) = runs[0]
        assert np.abs(E1).max() > 0
        for (E2, H2), (X2, p2) in runs[1:]:
            assert np.array_equal(E1, E2) and np.array_equal(H1, H2)
            assert np.array_equal(X1, X2) and np.array_equal(p1, p2)
    # a single periodic row (1-D planar problem) and a tiny periodic grid
    for n in ((96, 1), (5, 4)):
        out = []
        for fuse in (1, 2):
            s = gpu(n[0], n[1], 1, pol=pol, precision=prec, absorb=(20 if n[0] > 40 else 0, 0, 0),
                    sigma_max=W.SIGMA_MAX)
            s.set_source(8.0, [1.0, 0, 0], [0, 0, 1.0] if pol == "TM" else [0, 1.0, 0], 1.0, 1.0)
            s.set_fusion(fuse)
            s.step(70)
            out.append(s.fields())
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1]), n


def _mu_maps(nx, ny, W):
    """eps and mu blobs: a dielectric disc, a magnetic disc overlapping it, a
    matched (eps = mu) square and a magnetic strip reaching into the
    absorbing layer (where the incident-wave reference must switch off)."""
    y, x = np.mgrid[0:ny, 0:nx]
    eps = np.ones((1, ny, nx))
    mu = np.ones((1, ny, nx))
    eps[0][(x - 0.45 * nx) ** 2 + (y - 0.5 * ny) ** 2 < (0.15 * ny) ** 2] = 2.25
    mu[0][(x - 0.55 * nx) ** 2 + (y - 0.45 * ny) ** 2 < (0.12 * ny) ** 2] = 3.0
    sq = (abs(x - 0.7 * nx) < 4) & (abs(y - 0.7 * ny) < 4)
    eps[0][sq] = 1.7
    mu[0][sq] = 1.7
    mu[0][(y > ny - W - 4) & (x > 0.2 * nx) & (x < 0.3 * nx)] = 1.4
    return eps, mu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_permeability_fields_match_oracle(gpu, prec, pol):
    """Permeability map mu_r(x) (section 2.1: h_0^eq = (mu_r - 1) H,
    H = B / mu_r) on a ragged 83 x 61 grid absorbing on both axes, oblique
    incidence; eager steps and graph chunks mixed."""
    nx, ny, Wd = 83, 61, 10
    eps, mu = _mu_maps(nx, ny, Wd)
    th = np.deg2rad(30.0)
    kh = [np.cos(th), np.sin(th), 0.0]
    eh = [0, 0, 1.0] if pol == "TM" else [-np.sin(th), np.cos(th), 0.0]
    say("permeability", prec, pol)
    s, o = make_pair(gpu, nx, ny, 1, pol, prec, (Wd, Wd, 0), eps, 12.0, kh, eh, ramp=1.0)
    s.set_permeability(mu)
    o.set_mu(mu)
    for n in (1, 9, 190):
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"mu {pol} t={o.t}")
    # NULL map: back to mu_r = 1.  (Changing a map between steps re-slaves
    # the 2-D rest populations to the new map, which a literal run does not,
    # so compare from a restart.)
    s.set_permeability(None)
    s.reset()
    s2, o2 = make_pair(gpu, nx, ny, 1, pol, prec, (Wd, Wd, 0), eps, 12.0, kh, eh, ramp=1.0)
    s.step(90)
    o2.step(90)
    compare_fields(s, o2, prec, f"mu cleared {pol} t={o2.t}")
    s.close()
    s2.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_permeability_two_steps_bit_identical(gpu, prec, pol):
    """With a permeability map, two steps per launch (every tile) reproduce
    one step per launch bit for bit: fields and DFT phasors on a ragged grid,
    either axis periodic, odd step counts."""
    nx, ny = 203, 77
    rng = np.random.default_rng(8)
    eps = 1.0 + (rng.random((1, ny, nx)) < 0.2) * rng.uniform(0.2, 3.0, (1, ny, nx))
    mu = 1.0 + (rng.random((1, ny, nx)) < 0.2) * rng.uniform(0.2, 3.0, (1, ny, nx))
    mu[:, :4, :] = 1.6          # a magnetic strip inside the y layer
    th = np.deg2rad(25.0)
    kh = [np.cos(th), np.sin(th), 0.0]
    eh = [0, 0, 1.0] if pol == "TM" else [-np.sin(th), np.cos(th), 0.0]
    for absorb in ((11, 0, 0), (0, 9, 0)):
        runs = []
        for fuse, tile in [(1, (0, 0))] + [(2, t) for t in X2_TILES[prec]]:
            s = gpu(nx, ny, 1, pol=pol, precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
            s.set_permittivity(eps)
            s.set_permeability(mu)
            s.set_source(10.0, kh, eh, 1.0, 1.0)
            s.set_ntff((60, 20, 0), (140, 56, 0), 100, 30)
            s.set_fusion(fuse, tile)
            for n in (3, 131, 1):
                s.step(n)
            runs.append((s.fields(), s.phasors()))
            say("mu fusion", prec, pol, absorb, fuse, tile, s.t)
            s.close()
        (E1, H1), (X1, p1) = runs[0]
        assert np.abs(E1).max() > 0
        for (E2, H2), (X2, p2) in runs[1:]:
            assert np.array_equal(E1, E2) and np.array_equal(H1, H2)
            assert np.array_equal(X1, X2) and np.array_equal(p1, p2)


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_magnetic_cylinder_pipeline_intensity(gpu, pol):
    """Whole path on a magnetic-dielectric cylinder (eps 2, mu 1.5, 160^2,
    a = 9.5, lambda = 24, 1800 steps): contour phasors and |S|^2 against the
    oracle, FP64 and FP32."""
    case = W.cylinder_case(2.0, pol, n=160, a=9.5, lam=24.0, W=24, steps=1800, half=17.5)
    mu = W.circle(case.nx, case.radius, 1.5)
    inc_case = W.vacuum_companion(case)
    say("magnetic pipeline", pol)
    tot_o = run.run_2d(case, W.SIGMA_MAX, W.RAMP_PERIODS, mu=mu)
    inc_o = run.run_2d(inc_case, W.SIGMA_MAX, W.RAMP_PERIODS)
    th = np.arange(0, 360, 1.0)
    S_o = run.intensity_2d(case, tot_o, inc_o, th)
    for prec, ptol, stol in (("fp64", 1e-11, 1e-10), ("fp32", 1e-4, 1e-3)):
        kh, eh = W.plane_wave_2d(case.theta_deg, case.pol)
        tot_g = gpu(case.nx, case.ny, 1, pol=pol, precision=prec, absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        tot_g.set_permittivity(case.eps)
        tot_g.set_permeability(mu)
        tot_g.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        tot_g.set_ntff(case.box_lo, case.box_hi, *case.window)
        tot_g.step(case.steps)
        inc_g = _gpu_case(gpu, inc_case, prec)
        X, probe = tot_g.phasors()
        scale = np.abs(tot_o["phasors"]).max()
        perr = np.abs(X - tot_o["phasors"]).max() / scale
        say(pol, prec, "magnetic phasor err", perr)
        assert perr <= ptol
        S_g = tot_g.farfield(th, incident=inc_g)
        assert_intensity(S_g, S_o, stol, f"magnetic {pol} {prec}")


def test_permeability_api_limits(gpu):
    """What a permeability map refuses: batches, the adjoint, 3-D handles,
    values below 1; autotune with a map still verifies bit-identity."""
    from paper_2510_11042_amd import LbmEmError, step_many

    n = 64
    kh, eh = W.plane_wave_2d(0.0, "TM")
    s = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    s.set_source(16.0, kh, eh, 1.0, 1.0)
    assert s.get_fusion() == 2
    mu = np.ones((1, n, n))
    mu[0, 28:36, 28:36] = 2.0
    s.set_permeability(mu)
    assert s.get_fusion() == 2
    bad = mu.copy()
    bad[0, 0, 0] = 0.5
    with pytest.raises(LbmEmError):
        s.set_permeability(bad)
    other = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    other.set_source(16.0, kh, eh, 1.0, 1.0)
    other.set_fusion(1)
    with pytest.raises(LbmEmError):
        step_many([s, other], 2)
    s.step(10)
    ref = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    ref.set_source(16.0, kh, eh, 1.0, 1.0)
    ref.set_permeability(mu)
    ref.step(10)
    s.autotune(launches=2)
    assert s.t == 10
    s.step(30)
    ref.step(30)
    assert np.array_equal(s.fields()[0], ref.fields()[0]) and np.array_equal(s.fields()[1], ref.fields()[1])
    # the adjoint refuses a handle with a permeability map
    ref.set_ntff((20, 20, 0), (43, 43, 0), 48, 48)
    with pytest.raises(LbmEmError):
        ref.adjoint_setup(other, [0.0], (28, 28), (35, 35))
    s3 = gpu(8, 8, 8, pol="3D", precision="fp32", absorb=(0, 0, 0), sigma_max=W.SIGMA_MAX)
    with pytest.raises(LbmEmError):
        s3.set_permeability(np.ones((8, 8, 8)))
    for h in (s, other, ref, s3):
        h.close()


def _pec_disc(nx, ny, cx, cy, r):
    y, x = np.mgrid[0:ny, 0:nx]
    return (((x - cx) ** 2 + (y - cy) ** 2) < r * r)[None]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pec_fields_match_oracle(gpu, prec):
    """Perfect-conductor cells (zero-E reading) on a ragged 83 x 61 TM grid
    absorbing on both axes, with a conductor disc, a conductor strip reaching
    into the layer, a dielectric blob and a magnetic blob; oblique incidence,
    eager steps and graph chunks, the default two-step launches.  Then the
    conductor is removed (its cells return to mu_r = 1) and a restarted run is
    compared again."""
    nx, ny, Wd = 83, 61, 10
    eps, mu = _mu_maps(nx, ny, Wd)
    pec = _pec_disc(nx, ny, 0.3 * nx, 0.6 * ny, 7.5)
    pec[0, :4, 50:60] = True
    th = np.deg2rad(30.0)
    kh, eh = [np.cos(th), np.sin(th), 0.0], [0, 0, 1.0]
    say("pec", prec)
    s, o = make_pair(gpu, nx, ny, 1, "TM", prec, (Wd, Wd, 0), eps, 12.0, kh, eh, ramp=1.0)
    s.set_pec(pec)
    s.set_permeability(mu)          # the conductor stays
    o.set_mu(mu)
    o.set_pec(pec)
    for n in (1, 9, 190):
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"pec t={o.t}")
        Eg, _ = s.fields()
        assert np.all(Eg[pec] == 0.0)
    s.set_pec(None)
    s.reset()
    o2 = Oracle(nx, ny, 1, (Wd, Wd, 0), W.SIGMA_MAX)
    o2.set_eps(eps)
    mu2 = mu.copy()
    mu2[pec] = 1.0
    o2.set_mu(mu2)
    o2.set_source(12.0, kh, eh, 1.0, 1.0, [(nx - 1) / 2.0, (ny - 1) / 2.0, 0.0])
    s.step(90)
    o2.step(90)
    compare_fields(s, o2, prec, f"pec removed t={o2.t}")
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_pec_two_steps_bit_identical(gpu, prec):
    """Conductor cells through the two-step kernel (every tile) reproduce one
    step per launch bit for bit, TM, ragged grid, either axis periodic."""
    nx, ny = 203, 77
    pec = _pec_disc(nx, ny, 100.0, 38.0, 14.5)
    pec[0, :5, 20:40] = True                        # touches the y faces / layer
    th = np.deg2rad(25.0)
    kh, eh = [np.cos(th), np.sin(th), 0.0], [0, 0, 1.0]
    for absorb in ((11, 0, 0), (0, 9, 0)):
        runs = []
        for fuse, tile in [(1, (0, 0))] + [(2, t) for t in X2_TILES[prec]]:
            s = gpu(nx, ny, 1, pol="TM", precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
            s.set_pec(pec)
            s.set_source(10.0, kh, eh, 1.0, 1.0)
            s.set_ntff((60, 20, 0), (140, 56, 0), 100, 30)
            s.set_fusion(fuse, tile)
            for n in (3, 131, 1):
                s.step(n)
            runs.append((s.fields(), s.phasors()))
            say("pec fusion", prec, absorb, fuse, tile, s.t)
            s.close()
        (E1, H1), (X1, p1) = runs[0]
        assert np.abs(E1).max() > 0
        for (E2, H2), (X2, p2) in runs[1:]:
            assert np.array_equal(E1, E2) and np.array_equal(H1, H2)
            assert np.array_equal(X1, X2) and np.array_equal(p1, p2)


def test_pec_cylinder_pipeline_intensity(gpu):
    """Whole path on a PEC cylinder (160^2, a = 12.5, lambda = 24, TM, 1800
    steps): contour phasors and |S|^2 against the oracle, FP64 and FP32."""
    case = W.cylinder_case(1.0, "TM", n=160, a=12.5, lam=24.0, W=24, steps=1800, half=19.5)
    pec = W.circle(case.nx, case.radius, 2.0) > 1.0
    inc_case = W.vacuum_companion(case)
    say("pec pipeline")
    tot_o = run.run_2d(case, W.SIGMA_MAX, W.RAMP_PERIODS, pec=pec)
    inc_o = run.run_2d(inc_case, W.SIGMA_MAX, W.RAMP_PERIODS)
    th = np.arange(0, 360, 1.0)
    S_o = run.intensity_2d(case, tot_o, inc_o, th)
    for prec, ptol, stol in (("fp64", 1e-11, 1e-10), ("fp32", 1e-4, 1e-3)):
        kh, eh = W.plane_wave_2d(0.0, "TM")
        tot_g = gpu(case.nx, case.ny, 1, pol="TM", precision=prec, absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        tot_g.set_pec(pec)
        tot_g.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        tot_g.set_ntff(case.box_lo, case.box_hi, *case.window)
        tot_g.step(case.steps)
        inc_g = _gpu_case(gpu, inc_case, prec)
        X, probe = tot_g.phasors()
        scale = np.abs(tot_o["phasors"]).max()
        perr = np.abs(X - tot_o["phasors"]).max() / scale
        say(prec, "pec phasor err", perr)
        assert perr <= ptol
        S_g = tot_g.farfield(th, incident=inc_g)
        assert_intensity(S_g, S_o, stol, f"pec {prec}")


def test_pec_api_limits(gpu):
    """Conductor cells are refused on TE and 3-D handles; a handle with them
    is refused by batches and the adjoint."""
    from paper_2510_11042_amd import LbmEmError, step_many

    n = 64
    mask = _pec_disc(n, n, 31.5, 31.5, 5.0)
    te = gpu(n, n, 1, pol="TE", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    with pytest.raises(LbmEmError):
        te.set_pec(mask)
    s3 = gpu(8, 8, 8, pol="3D", precision="fp32", absorb=(0, 0, 0), sigma_max=W.SIGMA_MAX)
    with pytest.raises(LbmEmError):
        s3.set_pec(np.zeros((8, 8, 8), bool))
    kh, eh = W.plane_wave_2d(0.0, "TM")
    a = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    b = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    for h in (a, b):
        h.set_source(16.0, kh, eh, 1.0, 1.0)
    a.set_pec(mask)
    with pytest.raises(LbmEmError):
        step_many([a, b], 2)
    a.set_ntff((20, 20, 0), (43, 43, 0), 48, 48)
    with pytest.raises(LbmEmError):
        a.adjoint_setup(b, [0.0], (28, 28), (35, 35))
    a.set_pec(None)                 # no map left: batches work again
    step_many([a, b], 2)
    for h in (te, s3, a, b):
        h.close()


def _line_case(nx, ny, theta, pol):
    kh, eh = W.plane_wave_2d(theta, pol)
    return np.round(kh, 15), eh


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("theta,pol", [(0.0, "TM"), (90.0, "TE"), (180.0, "TE")])
def test_incident_line_fields_match_oracle(gpu, prec, theta, pol):
    """Exact incident line (layer rule that damps only the scattered part)
    on a ragged 83 x 61 grid absorbing on both axes with dielectric and
    magnetic blobs: fields every few steps and the line's phasors against
    the oracle's line, default two-step launches, eager and graph steps."""
    nx, ny, Wd = 83, 61, 10
    eps, mu = _mu_maps(nx, ny, Wd)
    kh, eh = _line_case(nx, ny, theta, pol)
    axis = 0 if abs(kh[0]) == 1.0 else 1
    say("line", prec, theta, pol)
    s, o = make_pair(gpu, nx, ny, 1, pol, prec, (Wd, Wd, 0), eps, 12.0, kh, eh, ramp=1.0)
    s.set_permeability(mu)
    o.set_mu(mu)
    lo, hi = (20, 15, 0), (62, 45, 0)
    s.set_ntff(lo, hi, 150, 36)
    cells = np.arange(nx * ny)
    o.set_dft(cells, 150, 36)
    s.set_incident_line(True)
    o.set_incident_line(axis)
    for n in (1, 9, 190):
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"line t={o.t}")
    Lg, Lo = s.line_phasors(), o.get_line_dft()
    err = np.abs(Lg - Lo).max() / np.abs(Lo).max()
    say("line phasors err", err)
    assert err <= (1e-11 if prec == "fp64" else 1e-4)
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_incident_line_reproduced_exactly(gpu, prec, pol):
    """A background-only grid with the incident line is the line at every
    row, bit for bit: its fields do not depend on y and its contour phasors
    equal the line's phasors at the node coordinates (one and two steps per
    launch)."""
    nx, ny = 150, 90
    kh, eh = W.plane_wave_2d(0.0, pol)
    for fuse in (1, 2):
        s = gpu(nx, ny, 1, pol=pol, precision=prec, absorb=(20, 12, 0), sigma_max=W.SIGMA_MAX)
        s.set_source(16.0, kh, eh, 1.0, 1.0)
        s.set_ntff((30, 25, 0), (110, 60, 0), 200, 48)
        s.set_incident_line(True)
        s.set_fusion(fuse)
        s.step(249)
        E, H = s.fields()
        assert np.abs(E).max() > 0.1
        assert np.array_equal(E, np.broadcast_to(E[:, :1], E.shape))
        assert np.array_equal(H, np.broadcast_to(H[:, :1], H.shape))
        X, probe = s.phasors()
        L = s.line_phasors()
        nodes = [(x, y) for y in range(25, 61) for x in range(30, 111)
                 if x in (30, 110) or y in (25, 60)]
        assert np.array_equal(X, L[[x for x, _ in nodes]])
        assert np.array_equal(probe, L[(30 + 110) // 2])
        s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_incident_line_two_steps_bit_identical(gpu, prec):
    """With the incident line, two steps per launch (every tile) reproduce
    one step per launch bit for bit, fields and phasors."""
    nx, ny = 203, 77
    rng = np.random.default_rng(9)
    eps = 1.0 + (rng.random((1, ny, nx)) < 0.2) * rng.uniform(0.2, 3.0, (1, ny, nx))
    eps[:, :, :12] = 1.0
    eps[:, :, -12:] = 1.0
    kh, eh = W.plane_wave_2d(0.0, "TM")
    runs = []
    for fuse, tile in [(1, (0, 0))] + [(2, t) for t in X2_TILES[prec]]:
        s = gpu(nx, ny, 1, pol="TM", precision=prec, absorb=(11, 9, 0), sigma_max=W.SIGMA_MAX)
        s.set_permittivity(eps)
        s.set_source(10.0, kh, eh, 1.0, 1.0)
        s.set_ntff((60, 20, 0), (140, 56, 0), 100, 30)
        s.set_incident_line(True)
        s.set_fusion(fuse, tile)
        for n in (3, 131, 1):
            s.step(n)
        runs.append((s.fields(), s.phasors(), s.line_phasors()))
        say("line fusion", prec, fuse, tile, s.t)
        s.close()
    (E1, H1), (X1, p1), L1 = runs[0]
    for (E2, H2), (X2, p2), L2 in runs[1:]:
        assert np.array_equal(E1, E2) and np.array_equal(H1, H2)
        assert np.array_equal(X1, X2) and np.array_equal(p1, p2) and np.array_equal(L1, L2)


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_incident_line_cylinder_intensity(gpu, pol):
    """|S|^2 with the incident line as the incident field (no companion run):
    against the oracle's line-based intensity (FP64 1e-10, FP32 1e-3) and
    against the GPU companion-based intensity (2e-4: the two differ only in
    how the layers force the incident wave)."""
    case = W.cylinder_case(2.25, pol, n=192, a=10.5, lam=32.0, W=32, steps=2400, half=19.5)
    kh, eh = W.plane_wave_2d(0.0, pol)
    th = np.arange(0, 360, 1.0)
    o = Oracle(case.nx, case.ny, 1, case.absorb, W.SIGMA_MAX)
    o.set_eps(case.eps)
    o.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
    nodes = ntff.box_nodes(case.box_lo, case.box_hi)
    pr = run.probe_node(case.box_lo, case.box_hi)
    cells = np.concatenate([ntff.linear_index(nodes, (case.nx, case.ny)),
                            ntff.linear_index(np.array([pr]), (case.nx, case.ny))])
    o.set_dft(cells, *case.window)
    o.set_incident_line(0)
    o.step(case.steps)
    X, Lx = o.get_dft(), o.get_line_dft()
    S_o = run.intensity_2d(case, {"nodes": nodes, "phasors": X[:-1], "probe": X[-1]},
                           {"phasors": Lx[nodes[:, 0]], "probe": Lx[pr[0]]}, th)
    for prec, stol in (("fp64", 1e-10), ("fp32", 1e-3)):
        s = gpu(case.nx, case.ny, 1, pol=pol, precision=prec, absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(case.eps)
        s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
        s.set_incident_line(True)
        s.step(case.steps)
        S_g = s.farfield(th)
        assert_intensity(S_g, S_o, stol, f"line {pol} {prec}")
        if prec == "fp32":
            tot = _gpu_case(gpu, case, prec)
            inc = _gpu_case(gpu, W.vacuum_companion(case), prec)
            S_c = tot.farfield(th, incident=inc)
            d = np.sqrt(np.mean((S_g - S_c) ** 2)) / S_c.max()
            say(pol, "line vs companion", d)
            assert d < 2e-4
        s.close()


def test_incident_line_api_limits(gpu):
    """The line needs a source along an axis (z in 3-D) and t = 0; a new
    source removes it; batches and the adjoint refuse a handle with one."""
    from paper_2510_11042_amd import LbmEmError, step_many

    n = 64
    s = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    with pytest.raises(LbmEmError):
        s.set_incident_line(True)                    # no source yet
    kh, eh = W.plane_wave_2d(30.0, "TM")
    s.set_source(16.0, kh, eh, 1.0, 1.0)
    with pytest.raises(LbmEmError):
        s.set_incident_line(True)                    # oblique
    kh, eh = W.plane_wave_2d(0.0, "TM")
    s.set_source(16.0, kh, eh, 1.0, 1.0)
    s.set_incident_line(True)
    other = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(12, 12, 0), sigma_max=W.SIGMA_MAX)
    other.set_source(16.0, kh, eh, 1.0, 1.0)
    with pytest.raises(LbmEmError):
        step_many([s, other], 2)
    s.set_ntff((20, 20, 0), (43, 43, 0), 48, 48)
    with pytest.raises(LbmEmError):
        s.adjoint_setup(other, [0.0], (28, 28), (35, 35))
    s.step(3)
    with pytest.raises(LbmEmError):
        s.set_incident_line(True)                    # t > 0
    s.set_source(16.0, kh, eh, 1.0, 1.0)             # removes the line
    with pytest.raises(LbmEmError):
        s.line_phasors()
    s.reset()
    s.set_incident_line(True)
    s.step(2)
    s3 = gpu(8, 8, 8, pol="3D", precision="fp32", absorb=(0, 0, 0), sigma_max=W.SIGMA_MAX)
    s3.set_source(4.0, [1.0, 0, 0], [0, 0, 1.0], 1.0, 1.0)
    with pytest.raises(LbmEmError):
        s3.set_incident_line(True)                   # 3-D lines run along z only
    for h in (s, other, s3):
        h.close()


@pytest.mark.parametrize("prec,nx", [("fp64", 800), ("fp32", 1600)])
def test_incident_line_long_line_matches_oracle(gpu, prec, nx):
    """A line too long for the LDS-resident line kernel (FP64 beyond 744
    cells, FP32 beyond 1489) takes the global-memory path, one or two steps
    per grid launch: fields against the oracle, eager steps and graph
    chunks, two steps per launch."""
    ny, Wd = 24, 6
    y, x = np.mgrid[0:ny, 0:nx]
    eps = np.ones((1, ny, nx))
    eps[0][((x - nx / 2) ** 2 + (y - ny / 2) ** 2) < 8 ** 2] = 2.5
    kh, eh = W.plane_wave_2d(0.0, "TM")
    say("long line", prec, nx)
    s, o = make_pair(gpu, nx, ny, 1, "TM", prec, (20, Wd, 0), eps, 12.0, kh, eh, ramp=1.0)
    s.set_incident_line(True)
    o.set_incident_line(0)
    for n in (1, 9, 140):
        s.step(n)
        o.step(n)
        compare_fields(s, o, prec, f"long line t={o.t}")
    s.close()


def test_measured_ceilings(gpu):
    """The measurement helpers: a plain copy and the multi-plane streaming
    pattern report positive bandwidths (below a generous bound on the HBM
    peak, above a floor any working device reaches) and refuse bad sizes
    with EINVAL."""
    import ctypes as C

    from paper_2510_11042_amd import _lib

    L = _lib.lib()
    g = C.c_double()
    assert L.lbm_em_copy_bandwidth(1 << 28, 3, C.byref(g)) == _lib.OK
    say("copy GB/s", g.value)
    assert 500.0 < g.value < 20000.0
    for nin, nout in ((24, 24), (28, 27), (1, 1), (32, 32)):
        g.value = 0.0
        assert L.lbm_em_stream_bandwidth(1 << 22, nin, nout, 3, C.byref(g)) == _lib.OK
        say("stream GB/s", nin, nout, g.value)
        assert 100.0 < g.value < 20000.0
    for cells, nin, nout, reps in ((0, 4, 4, 1), (1 << 20, 0, 0, 1), (1 << 20, 4, 5, 1), (1 << 20, 33, 4, 1),
                                   (1 << 20, 4, 4, 0), ((1 << 31) + 1, 4, 4, 1)):
        assert L.lbm_em_stream_bandwidth(cells, nin, nout, reps, C.byref(g)) == _lib.EINVAL
    assert L.lbm_em_stream_bandwidth(1 << 20, 4, 4, 1, None) == _lib.EINVAL


def test_edge_cases_and_errors(gpu):
    """Degenerate and invalid inputs: zero steps, negative steps, a 1 x 1
    periodic grid, empty or misplaced DFT windows and contours, the far field
    before its window ends, invalid permittivities."""
    from paper_2510_11042_amd import LbmEmError

    n = 48
    kh, eh = W.plane_wave_2d(0.0, "TM")
    s = gpu(n, n, 1, pol="TM", precision="fp32", absorb=(8, 8, 0), sigma_max=W.SIGMA_MAX)
    s.set_source(12.0, kh, eh, 1.0, 1.0)
    s.step(30)
    E0, H0 = s.fields()
    s.step(0)                                           # a no-op
    assert s.t == 30
    E1, H1 = s.fields()
    assert np.array_equal(E0, E1) and np.array_equal(H0, H1)
    with pytest.raises(LbmEmError):
        s.step(-1)
    with pytest.raises(LbmEmError):
        s.set_ntff((10, 10, 0), (30, 30, 0), 40, 0)     # empty window
    with pytest.raises(LbmEmError):
        s.set_ntff((0, 10, 0), (30, 30, 0), 40, 36)     # box touches the grid edge
    with pytest.raises(LbmEmError):
        s.set_ntff((10, 10, 0), (11, 30, 0), 40, 36)    # thinner than 3 nodes
    s.set_ntff((10, 10, 0), (37, 37, 0), 40, 36)
    with pytest.raises(LbmEmError):
        s.farfield([0.0, 90.0])                         # window not completed
    for bad in (0.5, np.nan, np.inf):
        eps = np.ones((1, n, n))
        eps[0, 5, 5] = bad
        with pytest.raises(LbmEmError):
            s.set_permittivity(eps)
    s.step(50)
    S = s.farfield([0.0, 90.0])                         # no incident: normalised by the amplitude
    assert np.all(np.isfinite(S))
    s.close()
    # a single periodic cell, no source: nothing moves, nothing is created
    one = gpu(1, 1, 1, pol="TE", precision="fp64", absorb=(0, 0, 0), sigma_max=W.SIGMA_MAX)
    one.step(65)
    E, H = one.fields()
    assert one.t == 65 and not np.any(E) and not np.any(H)
    one.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_incident_line_3d_matches_oracle(gpu, prec):
    """3-D incident line (incidence along +z): fields of a small dielectric
    sphere grid absorbing on all faces against the oracle with its line,
    one and two steps per launch, eager steps and graph chunks; then |S|^2
    from the line's phasors against the oracle's line-based intensity."""
    n = 48
    case = W.sphere_case(n=n, x_size=2.5, lam=12.0, eps_in=2.25, W=8, steps=360, half=8.5)
    say("3d line", prec)
    for fuse in (1, 2):
        s, o = make_pair(gpu, n, n, n, "3D", prec, (8, 8, 8), case.eps, case.lam, [0, 0, 1.0], [1.0, 0, 0],
                         ramp=1.0)
        s.set_incident_line(True)
        s.set_fusion(fuse)
        o.set_incident_line(2)
        for k in (1, 9, 130):
            s.step(k)
            o.step(k)
            compare_fields(s, o, prec, f"3d line fuse {fuse} t={o.t}")
        s.close()
    tot_o = run.run_3d(case, W.SIGMA_MAX, 1.0, line=True)
    L = tot_o["line"]
    pr = run.probe_node(case.box_lo, case.box_hi)
    inc_o = {"phasors": L[tot_o["nodes"][:, 2]], "probe": L[pr[2]]}
    s = gpu(n, n, n, pol="3D", precision=prec, absorb=(8, 8, 8), sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, 1.0)
    s.set_ntff(case.box_lo, case.box_hi, *case.window)
    s.set_incident_line(True)
    s.step(case.steps)
    th = np.arange(0, 180.01, 1.0)
    for phi in (0.0, 90.0):
        S_o = run.intensity_3d(case, tot_o, inc_o, th, np.full_like(th, phi))
        S_g = s.farfield(th, np.full_like(th, phi))
        assert_intensity(S_g, S_o, 1e-10 if prec == "fp64" else 1e-3, f"3d line phi {phi} {prec}")
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_incident_line_3d_exact_and_tiles(gpu, prec):
    """A background-only 3-D grid with the line is the line on every x-y
    plane, bit for bit; and every 3-D two-step tile reproduces one step per
    launch bit for bit with the line on a dielectric grid."""
    nx, ny, nz = 70, 36, 44
    s = gpu(nx, ny, nz, pol="3D", precision=prec, absorb=(6, 6, 8), sigma_max=W.SIGMA_MAX)
    s.set_source(10.0, [0, 0, -1.0], [0, 1.0, 0], 1.0, 1.0)
    s.set_incident_line(True)
    s.step(131)
    E, H = s.fields()
    assert np.abs(E).max() > 0.1
    assert np.array_equal(E, np.broadcast_to(E[:, :1, :1], E.shape))
    assert np.array_equal(H, np.broadcast_to(H[:, :1, :1], H.shape))
    s.close()
    rng = np.random.default_rng(13)
    eps = 1.0 + (rng.random((nz, ny, nx)) < 0.1) * rng.uniform(0.2, 2.0, (nz, ny, nx))
    runs = []
    for fuse, tile in [(1, (0, 0))] + [(2, t) for t in X3_TILES[prec]]:
        s = gpu(nx, ny, nz, pol="3D", precision=prec, absorb=(6, 6, 8), sigma_max=W.SIGMA_MAX)
        s.set_permittivity(eps)
        s.set_source(10.0, [0, 0, 1.0], [1.0, 0, 0], 1.0, 1.0)
        s.set_incident_line(True)
        s.set_fusion(fuse, tile)
        s.step(67)
        runs.append(s.fields())
        say("3d line fusion", prec, fuse, tile)
        s.close()
    for E2, H2 in runs[1:]:
        assert np.array_equal(runs[0][0], E2) and np.array_equal(runs[0][1], H2)


def test_incident_line_3d_limits(gpu):
    """A 3-D line needs incidence along z."""
    from paper_2510_11042_amd import LbmEmError

    s = gpu(16, 16, 16, pol="3D", precision="fp32", absorb=(4, 4, 4), sigma_max=W.SIGMA_MAX)
    s.set_source(8.0, [1.0, 0, 0], [0, 0, 1.0], 1.0, 1.0)
    with pytest.raises(LbmEmError):
        s.set_incident_line(True)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_incident_line_3d_global_memory_path(gpu, prec):
    """A 3-D line longer than the LDS holds (700 cells along z; FP32 LDS
    lines stop at 606, FP64 at 303) takes the global-memory path: a thin
    column (8 x 8 x 700, x and y periodic) with a dielectric slab against
    the oracle with its line, one and two steps per launch, eager steps and
    graph chunks, and a background-only column equal to the line bit for
    bit on every x-y plane."""
    nx, ny, nz = 8, 8, 700
    eps = np.ones((nz, ny, nx))
    eps[300:340, :, :] = 2.25
    eps[500:520, 2:6, 1:5] = 3.0
    for fuse in (1, 2):
        say("3d long line", prec, fuse)
        s, o = make_pair(gpu, nx, ny, nz, "3D", prec, (0, 0, 20), eps, 12.0, [0, 0, 1.0], [1.0, 0, 0], ramp=1.0)
        s.set_incident_line(True)
        s.set_fusion(fuse)
        o.set_incident_line(2)
        for k in (1, 9, 130, 600):
            s.step(k)
            o.step(k)
            compare_fields(s, o, prec, f"3d long line fuse {fuse} t={o.t}")
        s.close()
    s = gpu(nx, ny, nz, pol="3D", precision=prec, absorb=(0, 0, 20), sigma_max=W.SIGMA_MAX)
    s.set_source(12.0, [0, 0, -1.0], [0, 1.0, 0], 1.0, 1.0)
    s.set_incident_line(True)
    s.step(333)
    E, H = s.fields()
    assert np.abs(E).max() > 0.1
    assert np.array_equal(E, np.broadcast_to(E[:, :1, :1], E.shape))
    assert np.array_equal(H, np.broadcast_to(H[:, :1, :1], H.shape))
    s.close()
