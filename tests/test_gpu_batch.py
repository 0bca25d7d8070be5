"""Batched persistent stepping: many uneven 2-D instances advanced by one
launch per step must reproduce individually stepped handles bit for bit."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_11042_amd as P

    return P


def _make(P, case, prec, tile=None, fuse=2):
    kh, eh = W.plane_wave_2d(case.theta_deg, case.pol)
    s = P.Simulation(case.nx, case.ny, 1, pol=case.pol, precision=prec, absorb=case.absorb,
                     sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, kh, eh, 1.0, 1.0)
    if case.box_lo is not None:
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
    if tile:
        s.set_tile(*tile)
    s.set_fusion(fuse)
    return s


def _cases(seed, count, steps):
    """Seeded uneven scatterers (circle / hexagon, eps, size, lambda, angle)
    shrunk so the test stays small."""
    out = []
    sides = [160, 128, 96, 112, 144, 80, 136]
    for i, c in enumerate(W.batch_cases(count, seed=seed, W=12, steps=steps)):
        n = int(min(c.nx, sides[i % len(sides)]))
        lam = float(min(c.lam, 24.0))
        a = min(c.radius, n / 6)
        half = np.ceil(a) + 6.5
        cc = W.cylinder_case(c.eps_in, "TM", n=n, a=a, lam=lam, W=12, steps=steps, half=half,
                             theta_deg=c.theta_deg, shape=c.shape)
        out.append(cc)
    # one non-square grid too
    extra = W.cylinder_case(3.0, "TM", n=96, a=10.0, lam=12.0, W=12, steps=steps, half=16.5)
    extra.eps = extra.eps[:, :80, :]
    extra.ny = 80
    extra.box_lo, extra.box_hi = (31, 23, 0), (64, 56, 0)
    out.append(extra)
    return out


@pytest.mark.parametrize("prec,tile,fuse", [("fp32", None, 2), ("fp32", (4, 64, 4), 1), ("fp64", (2, 128, 2), 1),
                                             ("fp64", None, 2)])
def test_batch_equals_individual(lib, prec, tile, fuse):
    steps = 200                  # graph chunks, eager pairs and a trailing odd step
    cases = _cases(251011042, 6, steps)
    say("batch", prec, tile, fuse, [c.nx for c in cases])
    solo = [_make(lib, c, prec, tile, 1) for c in cases]
    for s in solo:
        s.step(steps)
    grouped = [_make(lib, c, prec, tile, fuse) for c in cases]
    b = lib.Batch(grouped)
    b.step(131)
    b.set_cache_budget(3 << 20)          # several groups from here on
    assert b.groups > 1
    b.step(69)
    for s, g in zip(solo, grouped):
        assert g.t == s.t == steps
        Es, Hs = s.fields()
        Eg, Hg = g.fields()
        assert np.array_equal(Es, Eg) and np.array_equal(Hs, Hg)
        Xs, ps = s.phasors()
        Xg, pg = g.phasors()
        assert np.array_equal(Xs, Xg) and np.array_equal(ps, pg)
    b.close()


def test_batch_routes_large_instances_to_their_own_kernels(lib):
    """An instance with at least one two-step tile per compute unit is
    advanced by the single-instance kernels as a group of its own; when its
    launch shape changes the batch re-plans it into the persistent launch.
    Either way every instance matches individual stepping bit for bit."""
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = 128
    while (n // 128) * (n // 32) < cus:
        n += 128
    steps = 200
    cases = _cases(91, 2, steps)
    big = W.cylinder_case(2.25, "TM", n=n, a=25.5, lam=32.0, W=32, steps=steps)
    cases.append(big)
    say("batch with a large instance", n, cus, [c.nx for c in cases])
    solo = [_make(lib, c, "fp32") for c in cases]
    for s in solo:
        s.step(steps)
    grouped = [_make(lib, c, "fp32") for c in cases]
    grouped[-1].set_fusion(2, (128, 32))
    b = lib.Batch(grouped)
    assert b.groups == 2                 # the two small instances, then the large one alone
    b.step(131)                          # graph chunks, an eager pair and an odd step
    grouped[-1].set_fusion(1)            # no longer eligible: re-planned into the batch
    b.step(69)
    assert b.groups == 1
    for s, g in zip(solo, grouped):
        assert g.t == s.t == steps
        Es, Hs = s.fields()
        Eg, Hg = g.fields()
        assert np.array_equal(Es, Eg) and np.array_equal(Hs, Hg)
        Xs, ps = s.phasors()
        Xg, pg = g.phasors()
        assert np.array_equal(Xs, Xg) and np.array_equal(ps, pg)
    b.close()


def test_batch_overlaps_large_instances_on_two_streams(lib):
    """Several instances on their own kernels run on two side streams of
    the batch; each still matches individual stepping bit for bit, and the
    batch's stream has joined them when the step call returns."""
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = 128
    while (n // 128) * (n // 32) < cus:
        n += 128
    steps = 200
    cases = [W.cylinder_case(e, "TM", n=n, a=25.5, lam=32.0, W=32, steps=steps) for e in (1.5, 2.25, 4.0)]
    cases.insert(1, _cases(13, 1, steps)[0])
    say("batch with three large instances", n, cus, [c.nx for c in cases])
    solo = [_make(lib, c, "fp32") for c in cases]
    for s in solo:
        s.step(steps)
    grouped = [_make(lib, c, "fp32") for c in cases]
    for g, c in zip(grouped, cases):
        if c.nx == n:
            g.set_fusion(2, (128, 32))
    b = lib.Batch(grouped)
    assert b.groups == 4
    b.step(131)
    b.step(69)
    for s, g in zip(solo, grouped):
        assert g.t == s.t == steps
        Es, Hs = s.fields()
        Eg, Hg = g.fields()
        assert np.array_equal(Es, Eg) and np.array_equal(Hs, Hg)
        Xs, ps = s.phasors()
        Xg, pg = g.phasors()
        assert np.array_equal(Xs, Xg) and np.array_equal(ps, pg)
    b.close()


def test_batch_autotune_keeps_state_and_results(lib):
    """Tuning the batch's tile changes no instance, and stepping with the
    chosen tile still reproduces individual stepping bit for bit (DFT
    window included)."""
    steps = 200
    cases = _cases(5, 4, steps)
    say("batch autotune", [c.nx for c in cases])
    solo = [_make(lib, c, "fp32") for c in cases]
    for s in solo:
        s.step(steps)
    grouped = [_make(lib, c, "fp32") for c in cases]
    b = lib.Batch(grouped)
    b.step(110)                          # tune mid-run, inside no DFT window yet
    before = [g.fields() for g in grouped]
    us = b.autotune(launches=3)
    assert us > 0
    # the batch reports the launch shape its tuner kept
    fuse, tile = b.tile()
    assert fuse == 2 and tile in [(64, 16), (128, 8), (128, 16), (256, 8), (256, 16), (128, 32)], (fuse, tile)
    for g, (E, H) in zip(grouped, before):
        assert g.t == 110
        E2, H2 = g.fields()
        assert np.array_equal(E, E2) and np.array_equal(H, H2)
    b.step(steps - 110)
    for s, g in zip(solo, grouped):
        assert g.t == s.t == steps
        assert np.array_equal(s.fields()[0], g.fields()[0]) and np.array_equal(s.fields()[1], g.fields()[1])
        Xs, ps = s.phasors()
        Xg, pg = g.phasors()
        assert np.array_equal(Xs, Xg) and np.array_equal(ps, pg)
    b.close()


def test_step_many_and_grid_size(lib):
    cases = _cases(7, 3, 90)
    say("step_many")
    solo = [_make(lib, c, "fp32") for c in cases]
    for s in solo:
        s.step(90)
    grouped = [_make(lib, c, "fp32") for c in cases]
    lib.step_many(grouped, 40)
    b = lib.Batch(grouped)
    b.set_grid(7)                                   # few blocks: each strides over many tiles
    b.step(50)
    for s, g in zip(solo, grouped):
        assert np.array_equal(s.fields()[0], g.fields()[0])


def test_batch_rejects_mismatched_handles(lib):
    from paper_2510_11042_amd import LbmEmError

    c = _cases(3, 2, 200)
    a = _make(lib, c[0], "fp32")
    b = _make(lib, c[1], "fp64")
    with pytest.raises(LbmEmError):
        lib.Batch([a, b])
    d = _make(lib, c[1], "fp32")
    d.step(1)
    with pytest.raises(LbmEmError):
        lib.step_many([a, d], 1)
    with pytest.raises(LbmEmError):
        lib.step_many([a, a], 1)
    # a handle held by a batch can be neither destroyed nor re-sourced
    g = [_make(lib, c[0], "fp32"), _make(lib, c[1], "fp32")]
    bb = lib.Batch(g)
    with pytest.raises(LbmEmError):
        g[0].close()
    with pytest.raises(LbmEmError):
        g[1].set_source(c[1].lam, [1.0, 0, 0], [0, 0, 1.0], 1.0, 1.0)
    bb.step(2)
    bb.close()
    g[1].set_source(c[1].lam, [1.0, 0, 0], [0, 0, 1.0], 1.0, 1.0)
    for s in g:
        s.close()


def _full_size(P, cases, prec="fp32"):
    out = []
    for c in cases:
        kh, eh = W.plane_wave_2d(c.theta_deg, c.pol)
        s = P.Simulation(c.nx, c.ny, 1, pol=c.pol, precision=prec, absorb=c.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(c.eps)
        s.set_source(c.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.set_ntff(c.box_lo, c.box_hi, *c.window)
        out.append(s)
    return out


@pytest.mark.parametrize("stress", [False, True])
def test_seeded_64_instance_batch_equals_individual(lib, stress):
    """The batched configuration at its real sizes: the 64 seeded instances
    (sides 256..448; with stress=True sides drawn from 256..1536, 70 M
    cells), the batch's own tuned tile, 330 steps (graph chunks, an odd
    tail, the DFT window at steps 231..329 or the instance's last period)
    against the same instances stepped one by one, bit for bit."""
    steps = 330
    cases = W.batch_cases(64, steps=steps, stress=stress)
    say("64-instance batch", "stress" if stress else "seeded", sum(c.nx * c.ny for c in cases))
    solo = _full_size(lib, cases)
    for s in solo:
        s.step(steps)
    grouped = _full_size(lib, cases)
    b = lib.Batch(grouped)
    b.autotune()
    say("groups", b.groups)
    b.step(steps - 1)
    b.step(1)
    for i, (s, g) in enumerate(zip(solo, grouped)):
        assert g.t == s.t == steps
        Es, Hs = s.fields()
        Eg, Hg = g.fields()
        assert np.array_equal(Es, Eg) and np.array_equal(Hs, Hg), i
        Xs, ps = s.phasors()
        Xg, pg = g.phasors()
        assert np.array_equal(Xs, Xg) and np.array_equal(ps, pg), i
        s.close()
    b.close()
    for g in grouped:
        g.close()
