#!/usr/bin/env python3
"""Benchmark of the electromagnetic lattice Boltzmann hot path on one MI355X.

One benchmark step = the 3-D dielectric-sphere workload (section 3.4):
a sphere of size parameter x = 6 at lambda = 24 cells (a = 22.92), eps_r =
2.25, plane wave along +z polarised along x, 24-cell absorbing layer, 4000
time steps with the last-period contour DFT, on a 384^3 and a 512^3 grid,
each with its eps_r = 1 companion run (the incident field), followed by the
near-to-far-field transform in the scattering planes phi = 0, 45 and 90
degrees at 0.5 degree resolution.  FP32 state and arithmetic, FP64 DFT
accumulators.  Inputs are resident in device memory before timing; the
state (2 x 6.1 GB and 2 x 14.5 GB per run) is far larger than the 256 MB
Infinity Cache, so the step kernel streams from HBM.

Reported value: lattice updates per second over the whole step (MLUPS).
roofline: the 3-D two-step kernel k_step3d_x2 against the 8 TB/s HBM peak,
counting each launch's minimal traffic: the state read and written once per
two time steps -- 27 scalars and eps (220 B) for a dielectric cell, the 24
moving scalars (192 B) for a vacuum cell, whose rest populations are
identically zero.  Extras: the 2-D cylinder job (1024^2, eight
solves, Infinity-Cache resident), two-stream and batched forms of it, the
sphere with the exact incident line instead of the companion, the
permeability and incident-line kernel variants, the batched configurations
(seeded and stress) and the inverse-design configuration.  cpu_baseline:
the FP64 oracle on a bounded sample of the sphere workload on the host
cores, with the GPU-vs-oracle field error on that sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline (fwd, adjoint, batched) at stated accuracy vs oracle"
HBM_PEAK_GBS = 8000.0
BYTES_2D = 11 * 4 * 2 + 4      # reduced 2-D state read + written, eps read (FP32)
BYTES_3D = 27 * 4 * 2 + 4      # dielectric cell: 27 scalars read + written, eps read (FP32)
BYTES_3D_VAC = 24 * 4 * 2      # vacuum cell: the 24 moving scalars (e_0 is identically zero)
CSRC = os.path.join(ROOT, "paper_2510_11042_amd", "csrc")
# the kernels and their launchers (the runtime lbm_em.hip is not hashed)
KERNEL_SOURCES = sorted(os.path.join("paper_2510_11042_amd", "csrc", f) for f in os.listdir(CSRC)
                        if f.endswith((".hpp", ".inc")) or (f.startswith("k_") and f.endswith(".hip")))


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(key, tile=None, field="bytes_per_launch"):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/) for
    `key` and (two-step kernels) the tile, or None when absent or taken on
    a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    if tile is not None:
        key = f"{key}_{tile[0]}x{tile[1]}"
    rec = json.load(open(path)).get(key)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get(field)


def cylinder_workload(Simulation, W, lbm_steps, tile=None, streams=None, precision="fp32"):
    """The eight solves; with `streams` = {pol: stream handle} each
    polarisation's instances are ordered on their own HIP stream."""
    sims = []
    for pol in ("TM", "TE"):
        for eps_in in (1.0, 1.5, 2.25, 4.0):
            case = W.cylinder_case(eps_in, pol, n=1024, steps=lbm_steps)
            if eps_in == 1.0:
                case = W.vacuum_companion(case)
            kh, eh = W.plane_wave_2d(0.0, pol)
            s = Simulation(1024, 1024, 1, pol=pol, precision=precision, absorb=case.absorb,
                           sigma_max=W.SIGMA_MAX, stream=streams[pol] if streams else None)
            s.set_permittivity(case.eps)
            s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
            s.set_ntff(case.box_lo, case.box_hi, *case.window)
            sims.append((pol, eps_in, s))
    # the library's autotuner picks the launch shape once per polarisation
    # (all instances share the grid); outside the timed region.  A given
    # two-step tile (profiling runs) replaces the tuning.
    for pol in ("TM", "TE"):
        group = [s for p, _, s in sims if p == pol]
        if tile is True:
            continue                  # the caller sets the tiles
        if tile:
            group[0].set_fusion(2, tile)
        else:
            group[0].autotune()
        for s in group[1:]:
            s.set_tile(*group[0].get_tile())
            s.set_fusion(group[0].get_fusion(), group[0].get_fusion_tile())
    return sims


def run_workload(sims, lbm_steps, theta, torch, events):
    """One benchmark step; appends (start, end) event pairs around stepping.
    Runs too short for the wave to reach the scatterer (profiling) skip the
    far field."""
    out = {}
    for pol, eps_in, s in sims:
        s.reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(lbm_steps)
        e1.record()
        events.append((e0, e1, lbm_steps))
    for pol in ("TM", "TE") if lbm_steps >= 2000 else ():
        inc = [s for p, e, s in sims if p == pol and e == 1.0][0]
        for p, e, s in sims:
            if p == pol and e != 1.0:
                out[(pol, e)] = s.farfield(theta, incident=inc)
    return out


def two_stream_extra(Simulation, W, torch, lbm_steps, theta, tiles):
    """The same eight solves with the TM instances on one HIP stream and the
    TE instances on a second one, enqueued alternately: two independent
    step kernels share the GPU and overlap each other's load, compute and
    store phases.  Whole job (stepping + far field), wall clock."""
    import ctypes as C

    st = {p: torch.cuda.Stream() for p in ("TM", "TE")}
    sims = cylinder_workload(Simulation, W, lbm_steps, streams={p: C.c_void_p(v.cuda_stream) for p, v in st.items()},
                             tile=None if tiles is None else True)
    if tiles is not None:
        for p, _, s in sims:
            s.set_fusion(2, tiles[p])
    tm = [s for p, _, s in sims if p == "TM"]
    te = [s for p, _, s in sims if p == "TE"]

    def job():
        for a, b in zip(tm, te):
            a.reset()
            b.reset()
            a.step(lbm_steps)
            b.step(lbm_steps)
        out = []
        for pol in ("TM", "TE"):
            inc = [s for p, e, s in sims if p == pol and e == 1.0][0]
            out += [s.farfield(theta, incident=inc) for p, e, s in sims if p == pol and e != 1.0]
        return out

    job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for _, _, s in sims:
        s.close()
    return {"workload": "the benchmark's eight solves + NTFF, TM and TE instances on two HIP streams",
            "MLUPS": len(sims) * 1024 * 1024 * lbm_steps / dt / 1e6, "seconds": dt}


def batched_job_extra(P, W, torch, lbm_steps, theta, tiles):
    """The same eight solves through the library's batches, one per
    polarisation: each instance fills the chip by itself, so the batch runs
    them on its own two-step kernels, alternating over two side streams
    where two independent kernels overlap.  Whole job (stepping + far
    field), wall clock."""
    sims = cylinder_workload(P.Simulation, W, lbm_steps, tile=None if tiles is None else True)
    if tiles is not None:
        for p, _, s in sims:
            s.set_fusion(2, tiles[p])
    batches = [P.Batch([s for p, _, s in sims if p == pol]) for pol in ("TM", "TE")]

    def job():
        for _, _, s in sims:
            s.reset()
        for b in batches:
            b.step(lbm_steps)
        out = []
        for pol in ("TM", "TE"):
            inc = [s for p, e, s in sims if p == pol and e == 1.0][0]
            out += [s.farfield(theta, incident=inc) for p, e, s in sims if p == pol and e != 1.0]
        return out

    job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    groups = [b.groups for b in batches]
    for b in batches:
        b.close()
    for _, _, s in sims:
        s.close()
    return {"workload": "the benchmark's eight solves + NTFF through two batches (TM, TE)",
            "groups": groups, "MLUPS": len(sims) * 1024 * 1024 * lbm_steps / dt / 1e6, "seconds": dt}


def sphere_job(Simulation, W, n, lbm_steps, tile=None, precision="fp32"):
    """The sphere (x = 6, lambda = 24, eps 2.25, W = 24) on an n^3 grid and
    its eps = 1 companion, contour DFT over the last period.  The launch
    shape is the library autotuner's pick for the sphere run (set up before
    timing; the companion takes the same), or `tile` for the two-step kernel."""
    case = W.sphere_case(n=n, steps=lbm_steps)
    case.n_dielectric = int(np.count_nonzero(case.eps != 1.0))
    sims = []
    for eps in (case.eps, None):
        s = Simulation(n, n, n, pol="3D", precision=precision, absorb=(case.W,) * 3, sigma_max=W.SIGMA_MAX)
        if eps is not None:
            s.set_permittivity(eps)
        s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
        if case.window[0] >= 0:          # runs shorter than a period (profiling) record no DFT
            s.set_ntff(case.box_lo, case.box_hi, *case.window)
        if tile:
            s.set_fusion(2, tile)
        elif eps is not None:
            s.autotune()
        else:
            s.set_tile(*sims[0].get_tile())
            s.set_fusion(sims[0].get_fusion(), sims[0].get_fusion_tile())
        sims.append(s)
    case.eps = None              # the map lives on the device now
    return case, sims


SPHERE_PHI = (0.0, 45.0, 90.0)


def launch_bytes_3d(n, n_dielectric):
    """Minimal bytes of one two-step launch of an n^3 grid with n_dielectric
    cells of eps_r != 1 (FP32)."""
    return (n ** 3 - n_dielectric) * BYTES_3D_VAC + n_dielectric * BYTES_3D


def run_sphere(jobs, lbm_steps, theta, torch, events):
    """One benchmark step over the sphere jobs; appends (start, end event,
    launches, cells, minimal bytes per launch averaged over the sphere and its
    companion) around the stepping of each grid size.  Runs too short for the
    DFT window (profiling) skip the far field."""
    out = {}
    for case, (tot, inc) in jobs:
        tot.reset()
        inc.reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tot.step(lbm_steps)
        inc.step(lbm_steps)
        e1.record()
        nb = 0.5 * (launch_bytes_3d(case.n, case.n_dielectric) + launch_bytes_3d(case.n, 0))
        events.append((e0, e1, 2 * lbm_steps // tot.get_fusion(), case.n ** 3, nb))
        # profiling runs too short for the wave to reach the sphere skip the far field
        if lbm_steps >= 1000 and lbm_steps >= case.window[0] + case.window[1]:
            for phi in SPHERE_PHI:
                out[(case.n, phi)] = tot.farfield(theta, np.full_like(theta, phi), incident=inc)
    return out


def sphere_line_extra(Simulation, W, torch, lbm_steps, theta):
    """The 384^3 sphere with the exact incident line (along z) instead of the
    companion run: one grid plus a line, whole job (stepping + far field)
    timed, and |S|^2 against the companion-run result."""
    n = 384
    case = W.sphere_case(n=n, steps=lbm_steps)
    s = Simulation(n, n, n, pol="3D", precision="fp32", absorb=(case.W,) * 3, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
    s.set_ntff(case.box_lo, case.box_hi, *case.window)
    s.set_incident_line(True)

    def job():
        s.reset()
        s.step(lbm_steps)
        return {phi: s.farfield(theta, np.full_like(theta, phi)) for phi in SPHERE_PHI}

    job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = job()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    return {"workload": f"sphere-{n}^3 with the incident line, {lbm_steps} steps + NTFF",
            "seconds": dt, "MLUPS": n ** 3 * lbm_steps / dt / 1e6}, S


def cylinder_extra(Simulation, W, torch, lbm_steps, theta, steps=2):
    """The 2-D circular-cylinder job (1024^2, a = 25.5, lambda = 32, W = 32,
    8000 steps, eps in {1.5, 2.25, 4.0} x {TM, TE} + two companions, 720
    angles).  Its state (2 x 46 MB + 4 MB per instance) sits in the 256 MB
    Infinity Cache: the bandwidth is the cache's, not HBM's."""
    sims = cylinder_workload(Simulation, W, lbm_steps)
    run_workload(sims, lbm_steps, theta, torch, [])
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(steps):
        run_workload(sims, lbm_steps, theta, torch, events)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    fuse = sims[0][2].get_fusion()
    step_ms = sum(a.elapsed_time(b) for a, b, _ in events)
    launches = sum(n for _, _, n in events) / fuse
    ms_per_launch = step_ms / launches
    cells = 1024 * 1024
    alg = cells * BYTES_2D
    kname = "k_step2d_x2" if fuse == 2 else "k_step2d"
    tiles = {p: list(s.get_fusion_tile()) for p, _, s in sims}
    res = {"workload": "cylinder-1024x1024-a25.5-lambda32-W32-8000steps-eps{1.5,2.25,4.0}x{TM,TE}"
                       "+vacuum-companions+NTFF720", "residency": "Infinity-Cache-resident (not HBM)",
           "instances": len(sims), "seconds_per_job": wall,
           "MLUPS": len(sims) * cells * lbm_steps / wall / 1e6, "kernel": kname, "tiles": tiles,
           "ms_per_launch": ms_per_launch, "algorithmic_bytes_per_launch": alg,
           "effective_cache_GBs": alg / (ms_per_launch * 1e-3) / 1e9,
           "traffic": recorded_traffic(f"{kname}_fp32_1024", tiles["TM"] if fuse == 2 else None)}
    for _, _, s in sims:
        s.close()
    return res, tiles if fuse == 2 else None


def magnetic_extra(Simulation, W, torch, steps=1600):
    """The two-step kernel's permeability variant on the cylinder grid: a
    magnetic-dielectric cylinder (eps 2, mu 1.5), TM, 1024^2; one more
    plane (mu) is read per launch: 96 B per cell."""
    case = W.cylinder_case(2.0, "TM", n=1024)
    mu = W.circle(case.nx, case.radius, 1.5)
    s = Simulation(case.nx, case.ny, 1, pol="TM", precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_permeability(mu)
    kh, eh = W.plane_wave_2d(0.0, "TM")
    s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
    s.step(256)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    fuse = s.get_fusion()
    ms = e0.elapsed_time(e1) / steps * fuse
    cells = case.nx * case.ny
    nbytes = cells * (BYTES_2D + 4)
    res = {"workload": "cylinder-1024x1024-eps2-mu1.5-TM", "kernel": "k_step2d_x2<float,TM,..,MU>" if fuse == 2
           else "k_step2d<float,TM,..,MU>", "steps_per_launch": fuse,
           "tile": list(s.get_fusion_tile()) if fuse == 2 else list(s.get_tile()),
           "ms_per_launch": ms, "MLUPS": cells * fuse / (ms * 1e-3) / 1e6,
           "algorithmic_bytes_per_launch": nbytes, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9}
    res["frac_of_hbm_peak"] = res["achieved_GBs"] / HBM_PEAK_GBS
    s.close()
    return res


def line_extra(Simulation, W, torch, steps=1600):
    """The cylinder grid with the exact incident line instead of a companion
    run: the line's own small launch precedes every grid launch, and the
    layer cells read the line's populations (1024^2, eps 2.25, TM)."""
    case = W.cylinder_case(2.25, "TM", n=1024)
    kh, eh = W.plane_wave_2d(0.0, "TM")
    out = {}
    for line in (False, True):
        s = Simulation(case.nx, case.ny, 1, pol="TM", precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(case.eps)
        s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        if line:
            s.set_incident_line(True)
        s.step(256)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        out["with_line" if line else "without"] = e0.elapsed_time(e1) / steps * 1e3
        s.close()
    res = {"workload": "cylinder-1024x1024-eps2.25-TM", "us_per_step": out,
           "line_overhead": out["with_line"] / out["without"] - 1.0,
           "note": "the line replaces the full vacuum companion run (one more grid of the same size)"}
    # the same on the 384^3 sphere (incidence along z)
    case = W.sphere_case(n=384, steps=200, with_eps=True)
    out3 = {}
    for line in (False, True):
        s = Simulation(384, 384, 384, pol="3D", precision="fp32", absorb=(case.W,) * 3, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(case.eps)
        s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
        if line:
            s.set_incident_line(True)
        s.step(64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(128)
        e1.record()
        torch.cuda.synchronize()
        out3["with_line" if line else "without"] = e0.elapsed_time(e1) / 128
        s.close()
    res["sphere_384_ms_per_step"] = out3
    res["sphere_line_overhead"] = out3["with_line"] / out3["without"] - 1.0
    return res


def batched_extra(P, W, torch, steps=6000, stress=False):
    """64 seeded uneven instances (circle/hexagon, eps, size, lambda, angle),
    6000 steps: one Batch (persistent launch per step, graph replay) against
    the same instances stepped one after another.  stress: sides drawn from
    256..1536 (70 M cells in all) instead of 256..448."""
    cases = W.batch_cases(64, steps=steps, stress=stress)
    sims = []
    for c in cases:
        kh, eh = W.plane_wave_2d(c.theta_deg, c.pol)
        s = P.Simulation(c.nx, c.ny, 1, pol=c.pol, precision="fp32", absorb=c.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(c.eps)
        s.set_source(c.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        if c.window[0] >= 0:             # runs shorter than a period (profiling) record no DFT
            s.set_ntff(c.box_lo, c.box_hi, *c.window)
        sims.append(s)
    cells = sum(c.nx * c.ny for c in cases)
    for s in sims:
        s.step(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.reset()
        s.step(steps)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    b = P.Batch(sims)
    tuned_us = b.autotune()         # the batch's own tile choice, outside the timed region
    for s in sims:
        s.reset()
    b.step(64)
    for s in sims:
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    fuse = sims[0].get_fusion()     # two steps per launch: the state moves once per two steps
    res = {"workload": f"64 seeded 2-D scatterers, sides {'256-1536' if stress else '256-448'}, {steps} steps",
           "cells": cells, "state_GB": cells * 2 * 11 * 4 / 1e9,
           "groups": b.groups, "MLUPS": cells * steps / t_batch / 1e6,
           "single_instance_MLUPS": cells * steps / t_single / 1e6, "steps_per_launch": fuse,
           "algorithmic_GBs": cells * steps / fuse * BYTES_2D / t_batch / 1e9}
    res["batched_over_single"] = res["MLUPS"] / res["single_instance_MLUPS"]
    res["autotune_us_per_step"] = tuned_us
    bfuse, btile = b.tile()
    res["tile"] = list(btile)
    # counter bytes of the batched kernel over a round of launches (every
    # group once) / the algorithmic bytes of that round, at the tile the
    # batch uses (profiles/, same kernel source)
    res["traffic_over_algorithmic"] = None if stress or bfuse != 2 else recorded_traffic(
        "k_step2d_x2_batch_fp32_seeded64", btile, field="traffic_over_algorithmic")
    b.close()
    for s in sims:
        s.close()
    return res


def adjoint_extra(P, W, torch, steps=6000):
    """Inverse design at 1024^2: J = sum |S|^2 over 10..20 degrees, 128^2
    design region; cost of the checkpointed forward and of the backward
    against a plain forward of the same length."""
    import numpy as np

    eps, (x0, y0) = W.design_region(1024, 128, seed=11042)
    case = W.cylinder_case(1.0, "TM", n=1024, steps=steps, half=72.5)
    kh, eh = W.plane_wave_2d(0.0, "TM")
    sims = []
    for e in (np.ones_like(eps), eps):
        s = P.Simulation(1024, 1024, 1, pol="TM", precision="fp32", absorb=case.absorb, sigma_max=W.SIGMA_MAX)
        s.set_permittivity(e)
        s.set_source(case.lam, kh, eh, 1.0, W.RAMP_PERIODS)
        s.set_ntff(case.box_lo, case.box_hi, *case.window)
        sims.append(s)
    inc, tot = sims
    inc.step(steps)
    tot.adjoint_setup(inc, np.arange(10.0, 20.01, 0.5), (x0, y0), (x0 + 127, y0 + 127))
    tot.forward_checkpointed(steps)
    tot.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot.reset()
    tot.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    J = tot.forward_checkpointed(steps)
    t_ck = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = tot.backward()
    t_bwd = time.perf_counter() - t0
    cells = 1024 * 1024
    res = {"workload": "inverse design 1024^2, 128^2 design, 6000 steps, J = sum |S|^2 10..20 deg",
           "J": J, "grad_norm": float(np.linalg.norm(g)), "forward_s": t_fwd, "forward_checkpointed_s": t_ck,
           "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
           "gradient_MLUPS": cells * steps / (t_ck + t_bwd) / 1e6,
           "checkpoints": int(np.ceil(steps / np.ceil(np.sqrt(steps))))}
    for s in sims:
        s.close()
    return res


def copy_ceiling(P):
    """The library's plain 16-byte-per-thread copy of 2 x 2 GiB: a measured
    bandwidth ceiling (read + written bytes)."""
    import ctypes as C

    from paper_2510_11042_amd import _lib

    g = C.c_double()
    _lib.check(_lib.lib().lbm_em_copy_bandwidth(2 ** 31, 10, C.byref(g)))
    return g.value


def stream_ceiling(P, n=384):
    """The library's multi-plane streaming kernel on an n^3 grid: 24 planes
    read and 24 written per cell (the 3-D two-step kernel's traffic for a
    vacuum cell) without the arithmetic; a measured ceiling for its access
    pattern (read + written bytes)."""
    import ctypes as C

    from paper_2510_11042_amd import _lib

    g = C.c_double()
    _lib.check(_lib.lib().lbm_em_stream_bandwidth(n ** 3, 24, 24, 10, C.byref(g)))
    return g.value


def host_cpu():
    """The host CPU's model name with its family / model / stepping numbers
    (virtual machines may report a generic name), and the thread count."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v
            elif info:
                break
    except OSError:
        pass
    model = info.get("model name", "unknown")
    ids = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    if ids:
        model += " (" + ", ".join(ids) + ")"
    return model, os.cpu_count()


def cpu_baseline(Simulation, W, target_s=20.0, n=384, S=None, n_dielectric=None):
    """FP64 oracle (literal 42-scalar scheme, OpenMP on all host threads) on
    a bounded sample of the benchmark workload: the 384^3 sphere, its first
    steps; the GPU (FP32, the benchmark's launch configuration) runs the
    same steps and its fields are compared with the oracle's.  With the
    timed step's |S|^2 (S, keyed by (grid, phi)) the accuracy gate also
    scores them against the Lorenz-Mie series of the oracle package, at the
    volume-equivalent radius of the staircase sphere."""
    import numpy as np

    from oracle import core as oracle_core
    from oracle import mie

    case = W.sphere_case(n=n, steps=4000)
    c = (n - 1) / 2.0
    t_alloc = time.perf_counter()
    o = oracle_core.Oracle(n, n, n, (case.W,) * 3, W.SIGMA_MAX)
    o.set_eps(case.eps)
    o.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS, [c, c, c])
    t_alloc = time.perf_counter() - t_alloc
    o.step(1)                     # the first step also faults in the state's pages
    t0 = time.perf_counter()
    o.step(1)
    per = time.perf_counter() - t0
    nsteps = int(max(2, min(400, target_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    o.step(nsteps)
    dt = time.perf_counter() - t0
    total = nsteps + 2
    s = Simulation(n, n, n, pol="3D", precision="fp32", absorb=(case.W,) * 3, sigma_max=W.SIGMA_MAX)
    s.set_permittivity(case.eps)
    s.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, W.RAMP_PERIODS)
    s.step(total)
    Eg, Hg = s.fields()
    s.close()
    Eo, Ho = o.fields()
    del o
    num = float(np.sum((Eg - Eo) ** 2) + np.sum((Hg - Ho) ** 2))
    den = float(np.sum(Eo ** 2) + np.sum(Ho ** 2))
    model, ncpu = host_cpu()
    field_err = float(np.sqrt(num / den)) if den > 0 else None
    gate = {"fields_vs_oracle_rel_l2": field_err, "fields_bound": 1e-4}
    if S:
        theta = np.arange(0.0, 180.01, 0.5)
        k = 2 * np.pi / case.lam
        nr = {}
        for (size, phi), s2 in S.items():
            a_eq = (n_dielectric[size] * 3 / (4 * np.pi)) ** (1 / 3)
            ref = mie.sphere_S2(theta, phi, k * a_eq, np.sqrt(case.eps_in))
            nr[f"{size}_phi{phi:g}"] = float(np.sqrt(np.mean((s2 - ref) ** 2)) / ref.max())
        gate["S2_vs_mie_nrms"] = nr
        gate["S2_bound"] = 2e-2
    gate["passed"] = bool(field_err is not None and field_err <= 1e-4 and
                          all(v <= 2e-2 for v in gate.get("S2_vs_mie_nrms", {}).values()))
    return {"value": n ** 3 * nsteps / dt / 1e6, "unit": "MLUPS", "cores": oracle_core.threads(),
            "kind": "oracle",
            "sample": f"eps 2.25 sphere {n}^3 (x = 6, lambda = 24, W = 24), steps 3..{total} of 4000 timed "
                      f"({dt:.1f} s; {41.7 * (n / 384) ** 3:.1f} GB of FP64 literal 42-scalar state, allocated "
                      f"in {t_alloc:.1f} s)",
            "host_cpu": model, "nproc": ncpu,
            "gpu_vs_oracle_rel_l2_fields": field_err,
            "sample_steps": total, "accuracy_gate": gate}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed benchmark steps")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lbm-steps", type=int, default=4000, help="time steps per solve (workload: 4000)")
    ap.add_argument("--sizes", default="384,512", help="sphere grid sizes (workload: 384,512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extras", default="copy,cylinder,streams,sphere_line,magnetic,line,batched,stress,adjoint",
                    help="comma list of extra measurements to run")
    ap.add_argument("--cylinder-steps", type=int, default=8000,
                    help="time steps of the 2-D cylinder extras (workload: 8000; fewer for profiling runs)")
    ap.add_argument("--batch-steps", type=int, default=6000,
                    help="time steps of the batched extras (workload: 6000; fewer for profiling runs)")
    ap.add_argument("--tile", default=None,
                    help="3-D two-step tile TX,TY instead of the default (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note, not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads as W
    from paper_2510_11042_amd import Simulation

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # the library's plain copy kernel k_copy16 on 2^30 bytes (read and
        # written once per launch), 1 warm-up + 3 timed launches
        import ctypes as C

        from paper_2510_11042_amd import _lib

        g = C.c_double()
        _lib.check(_lib.lib().lbm_em_copy_bandwidth(2 ** 30, 3, C.byref(g)))
        print(json.dumps({"kernel": "k_copy16", "bytes_read_per_launch": 2 ** 30,
                          "bytes_written_per_launch": 2 ** 30, "launches": 4, "GBs": g.value}))
        return 0
    sizes = [int(v) for v in args.sizes.split(",")]
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    theta = np.arange(0.0, 180.01, 0.5)
    jobs = [sphere_job(Simulation, W, n, args.lbm_steps, tile) for n in sizes]
    print(f"bench: sphere jobs {sizes} ready", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        run_sphere(jobs, args.lbm_steps, theta, torch, [])
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = run_sphere(jobs, args.lbm_steps, theta, torch, events)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"bench: {args.steps} timed steps in {wall:.1f} s", file=sys.stderr, flush=True)
    ms_per_step = wall * 1e3 / args.steps
    updates = sum(2 * case.n ** 3 * args.lbm_steps for case, _ in jobs)
    value = updates / (ms_per_step * 1e-3) / 1e6

    # the step kernel advances two time steps per launch (state read and
    # written once per launch): 192 B per vacuum cell and 220 B per
    # dielectric cell per launch are algorithmic
    tot0 = jobs[0][1][0]
    fuse = tot0.get_fusion()
    kname = "k_step3d_x2" if fuse == 2 else "k_step3d"
    per_size = {}
    for case, (tot, inc) in jobs:
        ev = [(a, b, n, nb) for a, b, n, c, nb in events if c == case.n ** 3]
        ms = sum(a.elapsed_time(b) for a, b, _, _ in ev) / sum(n for _, _, n, _ in ev)
        alg = ev[0][3]
        tl = list(tot.get_fusion_tile()) if fuse == 2 else list(tot.get_tile())
        per_size[str(case.n)] = {
            "ms_per_launch": ms, "algorithmic_bytes_per_launch": alg,
            "achieved_GBs": alg / (ms * 1e-3) / 1e9, "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "tile": tl, "MLUPS_per_instance": case.n ** 3 * fuse / (ms * 1e-3) / 1e6,
            "per_update_equivalent_GBs": alg * fuse / (ms * 1e-3) / 1e9,
            "full_state_GBs": case.n ** 3 * BYTES_3D / (ms * 1e-3) / 1e9,
            "traffic": recorded_traffic(f"{kname}_fp32_{case.n}", tl if fuse == 2 else None)}
    tot_ms = sum(a.elapsed_time(b) for a, b, _, _, _ in events)
    tot_bytes = sum(n * nb for _, _, n, _, nb in events)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    traffics = [per_size[k]["traffic"] for k in per_size]
    traffic = None
    if all(t is not None for t in traffics):
        # counter bytes over all launches of the step, per launch on average
        nl = {str(case.n): sum(n for _, _, n, c, _ in events if c == case.n ** 3) for case, _ in jobs}
        traffic = sum(per_size[k]["traffic"] * nl[k] for k in per_size) / sum(nl.values())
    line = {
        "metric": METRIC, "value": value, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "sphere-x6-lambda24-eps2.25-W24-" + "+".join(f"{n}^3" for n in sizes) +
                               f"-{args.lbm_steps}steps+vacuum-companions+NTFF-phi0/45/90-0.5deg",
                   "instances": 2 * len(sizes), "lbm_steps": args.lbm_steps,
                   "cells_per_instance": {str(n): n ** 3 for n in sizes}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname + "<float>", "steps_per_launch": fuse,
                     "per_size": per_size,
                     "frac_note": "achieved counts the launch's minimal traffic (the state read and written "
                                  "once per launch: 27 scalars and eps, 220 B, per dielectric cell; the 24 moving "
                                  "scalars, 192 B, per vacuum cell, whose rest populations are identically zero), "
                                  "summed over every launch of the timed steps and divided by their summed time "
                                  "(HIP events on the library's stream around each run; the figure includes the "
                                  "gaps between launches); per_update_equivalent_GBs counts those bytes per cell "
                                  "update; full_state_GBs counts 220 B per cell per launch",
                     "note": "state 2 x 6.1 GB (384^3) and 2 x 14.5 GB (512^3) per run: HBM-resident"},
    }
    for k, S in res.items():
        assert np.all(np.isfinite(S)) and S.max() > 0, k
    line["config"]["S2_forward_backward"] = {f"{n}_phi{phi:g}": [float(S[0]), float(S[-1])]
                                             for (n, phi), S in res.items()}
    for case, (tot, inc) in jobs:
        tot.close()
        inc.close()
    if not args.no_extra:
        import paper_2510_11042_amd as P

        want = set(args.extras.split(","))
        line["extra"] = {}
        say = lambda m: print(f"bench: extra {m}", file=sys.stderr, flush=True)
        if "copy" in want:
            line["roofline"]["measured_copy_GBs"] = copy_ceiling(P)
            line["roofline"]["measured_stream_24x24_GBs"] = stream_ceiling(P)
        th2 = np.arange(0.0, 360.0, 0.5)
        tiles = None
        cs = args.cylinder_steps
        if "cylinder" in want:
            say("cylinder")
            line["extra"]["cylinder_2d"], tiles = cylinder_extra(Simulation, W, torch, cs, th2)
        if "streams" in want:
            say("streams")
            line["extra"]["two_streams"] = two_stream_extra(Simulation, W, torch, cs, th2, tiles)
            line["extra"]["batched_job"] = batched_job_extra(P, W, torch, cs, th2, tiles)
        # the far field needs the incident wave at the sphere (profiling runs may be shorter)
        if "sphere_line" in want and 384 in sizes and args.lbm_steps >= 1000:
            say("sphere_line")
            r, S_line = sphere_line_extra(Simulation, W, torch, args.lbm_steps, theta)
            d = {}
            for phi in SPHERE_PHI:
                if (384, phi) in res:
                    ref = res[(384, phi)]
                    d[f"phi{phi:g}"] = float(np.sqrt(np.mean((S_line[phi] - ref) ** 2)) / ref.max())
            r["nrms_vs_companion_run"] = d
            line["extra"]["sphere_384_incident_line"] = r
        if "magnetic" in want:
            say("magnetic")
            line["extra"]["magnetic"] = magnetic_extra(Simulation, W, torch)
        if "line" in want:
            say("line")
            line["extra"]["incident_line"] = line_extra(Simulation, W, torch)
        if "batched" in want:
            say("batched")
            line["extra"]["batched"] = batched_extra(P, W, torch, steps=args.batch_steps)
        if "stress" in want:
            say("stress")
            line["extra"]["batched_stress"] = batched_extra(P, W, torch, steps=args.batch_steps, stress=True)
        if "adjoint" in want:
            say("adjoint")
            line["extra"]["adjoint"] = adjoint_extra(P, W, torch)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(Simulation, W, S=res,
                                            n_dielectric={case.n: case.n_dielectric for case, _ in jobs})
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
