"""Write the stored oracle results that the full-length GPU parity tests read.

TEST INFRASTRUCTURE.  Calls only the FP64 oracle (oracle/) and the seeded
input generators (workloads/); nothing here comes from the HIP library.

  python tests/golden/make_golden.py cylinder   -> cylinder1024_8000.npz
  python tests/golden/make_golden.py batch      -> batch_instances_6000.npz

cylinder: the 2-D circular-cylinder workload at its full size (1024^2,
a = 25.5, lambda = 32, W = 32, 8000 steps, DFT over the last period
7904..7999, section 2.4) for eps_r in {1.5, 2.25, 4.0}, TM and TE, and the
eps_r = 1 companion run of each polarisation (the incident field, section
2.1's subtraction).  Stored per run: the contour phasors and the probe
phasor; per scatterer |S(theta)|^2 at 720 angles (0.5 degree steps from
the incidence direction, Eq. S2D); for eps_r = 2.25 and the companions the
final fields (step 8000) on fixed rows and columns through the scatterer.

batch: two instances of the seeded 64-instance batch (a hexagon at 10.9
degrees and an oblique circle at 53.9 degrees), 6000 steps, with their
companions: phasors, |S|^2 and final fields on rows and columns through the
scatterer.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import run  # noqa: E402

THETA = np.arange(0.0, 360.0, 0.5)
# rows and columns of the stored field snapshots (1024^2 grid): the layers,
# the gap between layer and contour, the contour, the scatterer's interior
CYL_LINES = (16, 200, 478, 500, 511, 512, 523, 545, 800, 1010)
BATCH_IDS = (1, 2)


def field_lines(E, H, lines, comps):
    """(len(lines), 2, n, len(comps)) float64: row y = l and column x = l of
    the field components comps (0..2 of E, 3..5 of H)."""
    F = np.concatenate([E[0], H[0]], axis=-1)[..., list(comps)]   # (ny, nx, c)
    rows = np.stack([F[l, :, :] for l in lines])
    cols = np.stack([F[:, l, :] for l in lines])
    return np.stack([rows, cols], axis=1)


def pol_comps(pol):
    return (2, 3, 4) if pol == "TM" else (0, 1, 5)


def solve(case, fields_lines=None):
    t0 = time.perf_counter()
    r = run.run_2d(case, W.SIGMA_MAX, W.RAMP_PERIODS, collect_fields=fields_lines is not None)
    out = {"phasors": r["phasors"], "probe": r["probe"]}
    if fields_lines is not None:
        out["fields"] = field_lines(r["E"], r["H"], fields_lines, pol_comps(case.pol))
    print(f"  {case.name} {case.pol} eps {case.eps_in:g}: {time.perf_counter() - t0:.0f} s", flush=True)
    return out


def make_cylinder(path):
    data = {"theta_rel_deg": THETA, "lines": np.array(CYL_LINES), "steps": np.array(8000)}
    for pol in ("TM", "TE"):
        base = W.cylinder_case(2.25, pol, n=1024, steps=8000)
        inc = solve(W.vacuum_companion(base), CYL_LINES)
        for k, v in inc.items():
            data[f"{pol}_vac_{k}"] = v
        for eps_in in (1.5, 2.25, 4.0):
            case = W.cylinder_case(eps_in, pol, n=1024, steps=8000)
            tot = solve(case, CYL_LINES if eps_in == 2.25 else None)
            tag = f"{pol}_eps{eps_in:g}"
            for k, v in tot.items():
                data[f"{tag}_{k}"] = v
            data[f"{tag}_S2"] = run.intensity_2d(case, {**tot, "nodes": _nodes(case)},
                                                 {**inc, "nodes": _nodes(case)}, THETA)
    np.savez_compressed(path, **data)


def _nodes(case):
    from oracle import ntff

    return ntff.box_nodes(case.box_lo, case.box_hi)


def make_batch(path):
    cases = W.batch_cases(64)
    data = {"theta_rel_deg": THETA, "ids": np.array(BATCH_IDS)}
    for i in BATCH_IDS:
        case = cases[i]
        c = (case.nx - 1) / 2.0
        lines = tuple(sorted({20, int(c) - int(case.radius) - 3, int(c), int(c) + 1,
                              int(c) + int(case.radius) // 2, case.nx - 40}))
        data[f"b{i}_lines"] = np.array(lines)
        inc = solve(W.vacuum_companion(case), lines)
        tot = solve(case, lines)
        for k, v in inc.items():
            data[f"b{i}_vac_{k}"] = v
        for k, v in tot.items():
            data[f"b{i}_{k}"] = v
        data[f"b{i}_S2"] = run.intensity_2d(case, {**tot, "nodes": _nodes(case)},
                                            {**inc, "nodes": _nodes(case)}, THETA)
    np.savez_compressed(path, **data)


if __name__ == "__main__":
    what = sys.argv[1:] or ["cylinder", "batch"]
    for w in what:
        out = os.path.join(HERE, {"cylinder": "cylinder1024_8000.npz", "batch": "batch_instances_6000.npz"}[w])
        print(w, "->", out, flush=True)
        {"cylinder": make_cylinder, "batch": make_batch}[w](out)
