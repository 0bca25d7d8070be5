"""The 3-D two-step z march at the sizes the benchmark runs.

* 384^3 and 512^3 spheres (x = 6 at lambda = 24, eps 2.25, W = 24) in the
  launch configuration the benchmark times (the autotuner's pick: two
  steps per launch, 128 x 8 tiles at 384^3 and a wider tile at 512^3, z
  chunks chosen for the device): bit-identical to one step per launch over
  three graph chunks (the first outside the DFT window, so it replays the
  kernels without the contour accumulation) and an odd trailing step,
  fields and contour phasors.
* A 512-thread tile whose chunk is longer than its block (512^3, 128 x 4):
  two steps per launch against one, with dielectric slabs that carry
  fields on planes far apart in the chunk.
* FP64 and FP32 against the oracle on a 160 x 96 x 128 grid, where the
  default tile leaves ragged x tiles and the z march takes several chunks.
* A permittivity map changed between steps, against the oracle: the 3-D
  state keeps the rest populations e_0 as the literal scheme does, so cells
  that leave the dielectric keep theirs (the two-step kernel must not treat
  their planes as vacuum) and cells that enter it start from zero.
"""
import numpy as np
import pytest

import workloads as W
from oracle.core import Oracle
from paritycheck import max_rel, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Sim():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11042_amd import Simulation

    return Simulation


def _sphere_sim(Sim, case, prec="fp32"):
    n = case.n
    s = Sim(n, n, n, pol="3D", precision=prec, absorb=(case.W,) * 3, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
    return s


@pytest.mark.parametrize("n", [384, 512])
def test_sphere_two_steps_per_launch_bit_identical(Sim, n):
    case = W.sphere_case(n=n, steps=195)
    runs = []
    for fuse in (2, 1):
        s = _sphere_sim(Sim, case)
        # a contour through the forced layers (the wave is there from the
        # start), window [100, 172): graph chunk [0, 64) lies before it
        s.set_ntff((8, 8, 8), (n - 9, n - 9, n - 9), 100, 72)
        if fuse == 2:
            rec = s.autotune()
            assert rec["fusion"] == 2, rec
        else:
            s.set_fusion(1)
        say(f"{n}^3 fusion", s.get_fusion(), s.get_fusion_tile())
        for k in (64, 128, 3):
            s.step(k)
        assert s.t == 195
        E, H = s.fields()
        X, p = s.phasors()
        runs.append((E, H, X, p))
        s.close()
    (E2, H2, X2, p2), (E1, H1, X1, p1) = runs
    assert np.abs(E1).max() > 0 and np.abs(X1).max() > 0
    assert np.array_equal(E1, E2) and np.array_equal(H1, H2)
    assert np.array_equal(X1, X2) and np.array_equal(p1, p2)


def test_long_chunk_vacuum_flags_bit_identical(Sim):
    """A 512-thread tile marching a chunk longer than its block: on a
    256-CU device the 512^3 grid with 128 x 4 tiles takes a single chunk of
    512 planes, so the block forms the planes' vacuum flags in two passes
    and they span nine 64-bit words.  Dielectric slabs against the forced x
    layer, on planes in several of those words, carry fields from the first
    steps (a bug in the flags would treat them as vacuum).  Two steps per
    launch against one, bit for bit."""
    n, Wl = 512, 24
    eps = np.ones((n, n, n))
    slabs = (30, 100, 300, 505)
    for z0 in slabs:
        eps[z0:z0 + 6, :, Wl:Wl + 6] = 2.25
    runs = []
    for fuse, tile in ((2, (128, 4)), (1, (0, 0))):
        s = Sim(n, n, n, pol="3D", precision="fp32", absorb=(Wl,) * 3, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(eps)
        s.set_source(24.0, [0, 0, 1.0], [1.0, 0, 0], 1.0, 1.0)
        s.set_fusion(fuse, tile)
        say("512^3 long chunk, fusion", s.get_fusion(), s.get_fusion_tile())
        for k in (64, 3):
            s.step(k)
        runs.append(s.fields())
        s.close()
    (E2, H2), (E1, H1) = runs
    for z0 in slabs:
        assert np.abs(E1[z0:z0 + 6, :, Wl:Wl + 6]).max() > 0, z0
    assert np.array_equal(E1, E2) and np.array_equal(H1, H2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multichunk_ragged_grid_vs_oracle(Sim, prec):
    nx, ny, nz = 160, 96, 128
    steps = 150
    eps = np.ones((nz, ny, nx))
    z, y, x = np.ogrid[0:nz, 0:ny, 0:nx]
    eps[(x - 80.5) ** 2 + (y - 47.5) ** 2 + (z - 60.0) ** 2 < 14.0 ** 2] = 2.25
    eps[(x - 120.0) ** 2 / 4 + (y - 30.0) ** 2 + (z - 90.0) ** 2 < 8.0 ** 2] = 3.0
    k3 = np.array([0.3, 0.2, 1.0]) / np.linalg.norm([0.3, 0.2, 1.0])
    e3 = np.cross(k3, [0.0, 1.0, 0.0])
    e3 /= np.linalg.norm(e3)
    absorb = (12, 12, 12)
    lam = 12.0
    say("multichunk", prec)
    o = Oracle(nx, ny, nz, absorb, W.SIGMA_MAX)
    o.set_eps(eps)
    o.set_source(lam, k3, e3, 1.0, 1.0, [(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    o.step(steps)
    Eo, Ho = o.fields()
    s = Sim(nx, ny, nz, pol="3D", precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(eps)
    s.set_source(lam, k3, e3, 1.0, 1.0)
    say("tile", s.get_fusion(), s.get_fusion_tile())
    assert s.get_fusion() == 2
    s.step(steps)
    Eg, Hg = s.fields()
    # the wave has reached the first scatterer
    assert np.abs(Eo[45:75, 35:60, 68:94]).max() > 0.1
    if prec == "fp64":
        err = max(max_rel(Eg, Eo), max_rel(Hg, Ho))
        say("fp64 max rel", err)
        assert err <= 1e-12
    else:
        err = rel_l2(np.concatenate([Eg.ravel(), Hg.ravel()]), np.concatenate([Eo.ravel(), Ho.ravel()]))
        say("fp32 rel L2", err)
        assert err <= 1e-4
    s.close()


@pytest.mark.parametrize("order,prec", [("leave", "fp64"), ("enter", "fp64"), ("leave", "fp32")])
def test_permittivity_change_between_steps_vs_oracle(Sim, order, prec):
    nx, ny, nz = 72, 40, 48
    absorb = (8, 8, 8)
    lam = 10.0
    steps1, steps2 = 90, 60
    z, y, x = np.ogrid[0:nz, 0:ny, 0:nx]
    blob = np.ones((nz, ny, nx))
    blob[(x - 30.0) ** 2 + (y - 20.0) ** 2 + (z - 24.0) ** 2 < 7.0 ** 2] = 2.5
    vac = np.ones((nz, ny, nx))
    first, second = (blob, vac) if order == "leave" else (vac, blob)
    k3, e3 = [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]
    centre = [(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0]
    say("eps change", order, prec)
    o = Oracle(nx, ny, nz, absorb, W.SIGMA_MAX)
    o.set_eps(first)
    o.set_source(lam, k3, e3, 1.0, 1.0, centre)
    o.step(steps1)
    if order == "leave":
        # the dielectric holds rest populations e_0 (population 0, the
        # first three components) when its map is removed
        e0 = o.get_state()[..., 0, 0:3]
        assert np.abs(e0).max() > 1e-3
    o.set_eps(second)
    o.step(steps2)
    Eo, Ho = o.fields()
    s = Sim(nx, ny, nz, pol="3D", precision=prec, absorb=absorb, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(first)
    s.set_source(lam, k3, e3, 1.0, 1.0)
    assert s.get_fusion() == 2
    s.step(steps1)
    s.set_permittivity(second)
    s.step(steps2)
    Eg, Hg = s.fields()
    assert np.abs(Eo[17:32, 13:28, 23:38]).max() > 0.1
    if prec == "fp64":
        err = max(max_rel(Eg, Eo), max_rel(Hg, Ho))
        say("fp64 max rel", err)
        assert err <= 1e-12
    else:
        err = rel_l2(np.concatenate([Eg.ravel(), Hg.ravel()]), np.concatenate([Eo.ravel(), Ho.ravel()]))
        say("fp32 rel L2", err)
        assert err <= 1e-4
    s.close()
