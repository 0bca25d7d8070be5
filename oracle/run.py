"""Drive whole scattering runs through the oracle.

TEST INFRASTRUCTURE ONLY.

A run follows the paper's procedure (sections 2.3-2.4): step the scheme to
a steady state, DFT the fields on a closed contour over the last period,
subtract the incident field, transform to the far field.  The incident
field is taken from a companion run with eps = 1 everywhere and identical
grid, layers, source and window (reading: this cancels the lattice
dispersion of the incident wave exactly); its phasor at the centre node of
the contour is the incident amplitude "in the vicinity of the scatterer"
of Eq. S2D / S3D.
"""
import numpy as np

from . import ntff
from .core import Oracle


def probe_node(lo, hi):
    return tuple((l + h) // 2 for l, h in zip(lo, hi))


def run_2d(case, sigma_max, ramp_periods, steps=None, collect_fields=False, mu=None, pec=None):
    """Run a workloads.Case2D (mu: optional permeability map, pec: optional
    perfect-conductor mask, both shaped like case.eps); returns dict(nodes,
    phasors (p, 6), probe (6,), E, H (final fields, optional))."""
    steps = case.steps if steps is None else steps
    o = Oracle(case.nx, case.ny, 1, case.absorb, sigma_max)
    o.set_eps(case.eps)
    if mu is not None:
        o.set_mu(mu)
    if pec is not None:
        o.set_pec(pec)
    from workloads import plane_wave_2d

    kh, eh = plane_wave_2d(case.theta_deg, case.pol)
    o.set_source(case.lam, kh, eh, 1.0, ramp_periods)
    out = {}
    if case.box_lo is not None:
        nodes = ntff.box_nodes(case.box_lo, case.box_hi)
        pr = probe_node(case.box_lo, case.box_hi)
        cells = np.concatenate([ntff.linear_index(nodes, (case.nx, case.ny)),
                                ntff.linear_index(np.array([pr]), (case.nx, case.ny))])
        w0, wl = case.window
        o.set_dft(cells, w0, wl)
        out["nodes"] = nodes
    o.step(steps)
    if case.box_lo is not None:
        X = o.get_dft()
        out["phasors"] = X[:-1]
        out["probe"] = X[-1]
    if collect_fields:
        out["E"], out["H"] = o.fields()
    out["oracle"] = o
    return out


def intensity_2d(case, total, incident, theta_rel_deg):
    """|S(theta)|^2 with theta measured from the incidence direction."""
    k = 2 * np.pi / case.lam
    Xs = total["phasors"] - incident["phasors"]
    center = ((case.nx - 1) / 2.0, (case.ny - 1) / 2.0)
    if case.pol == "TM":
        amp = incident["probe"][2]              # E_z
    else:
        amp = incident["probe"][5]              # H_z
    th = np.asarray(theta_rel_deg, dtype=float) + case.theta_deg
    return ntff.farfield_2d(total["nodes"], Xs[:, :3], Xs[:, 3:], case.box_lo, case.box_hi, k,
                            th, case.pol, center, amp)


def run_3d(case, sigma_max, ramp_periods, eps=None, steps=None, line=False):
    """Sphere-type 3-D run: k along +z, E along +x (section 3.4); line: with
    the exact incident line (its phasors returned as "line")."""
    steps = case.steps if steps is None else steps
    n = case.n
    W = case.W
    o = Oracle(n, n, n, (W, W, W), sigma_max)
    o.set_eps(case.eps if eps is None else eps)
    o.set_source(case.lam, [0, 0, 1.0], [1.0, 0, 0], 1.0, ramp_periods)
    nodes = ntff.box_nodes(case.box_lo, case.box_hi)
    pr = probe_node(case.box_lo, case.box_hi)
    cells = np.concatenate([ntff.linear_index(nodes, (n, n, n)),
                            ntff.linear_index(np.array([pr]), (n, n, n))])
    w0, wl = case.window
    o.set_dft(cells, w0, wl)
    if line:
        o.set_incident_line(2)
    o.step(steps)
    X = o.get_dft()
    out = {"nodes": nodes, "phasors": X[:-1], "probe": X[-1], "oracle": o}
    if line:
        out["line"] = o.get_line_dft()
    return out


def intensity_3d(case, total, incident, theta_deg, phi_deg):
    k = 2 * np.pi / case.lam
    Xs = total["phasors"] - incident["phasors"]
    c = (case.n - 1) / 2.0
    return ntff.farfield_3d(total["nodes"], Xs[:, :3], Xs[:, 3:], case.box_lo, case.box_hi, k,
                            theta_deg, phi_deg, (c, c, c), incident["probe"][0])


def normalized_rms(S, ref):
    """Normalized RMS error of section 3.2, Eq. rms_error."""
    S, ref = np.asarray(S), np.asarray(ref)
    return float(np.sqrt(np.mean((S - ref) ** 2)) / np.max(ref))
