"""Near-to-far-field transform of recorded phasors -> |S|^2 (FP64).

TEST INFRASTRUCTURE ONLY.

Follows section 2.4 (equivalence principle after Schneider / Taflove):
  - phasors of E and H on a closed fictitious boundary, obtained by a DFT
    of one steady-state period (exp(+j omega t) convention);
  - equivalent currents J = n x H, M = -n x E (n the outward normal);
  - 2-D potentials with H_0^(2)(k|r - r'|), 3-D with exp(-jkR)/(4 pi R),
    the factor 3 of the lattice units combining with omega = k/3 so that
    the background medium has unit impedance;
  - radiated far field from the potentials, and the angular intensity of
    section 2.3 (Eq. S2D: k r |E_s|^2/|E_i|^2, Eq. S3D: k^2 r^2 |E_s|^2/|E_i|^2).

Far-field limits used (r -> infinity, background eps = mu = 1):
  2-D, with N = sum w J e^{jk rhat.r'}, L = sum w M e^{jk rhat.r'}:
      E_z = (k/4) C [-N_z + (rhat x L)_z],  H_z = -(k/4) C [L_z + (rhat x N)_z],
      C = sqrt(2j/(pi k r)) e^{-jkr}, so
      |S|^2_TM = k^2/(8 pi) |N_z - (rhat x L)_z|^2 / |E_i|^2
      |S|^2_TE = k^2/(8 pi) |L_z + (rhat x N)_z|^2 / |H_i|^2
  3-D:
      E_theta = -jk G (N_theta + L_phi),  E_phi = -jk G (N_phi - L_theta),
      G = e^{-jkr}/(4 pi r), so
      |S|^2 = k^4/(16 pi^2) (|N_theta + L_phi|^2 + |N_phi - L_theta|^2) / |E_i|^2

Contour reading (the paper does not fix it): an axis-aligned box through
node centres, every edge (2-D) or face (3-D) integrated on its own with the
trapezoid rule (unit spacing, half weight on end nodes), so corner and edge
nodes contribute once per edge/face with that edge's/face's normal.
"""
import numpy as np


# ---------------------------------------------------------------------------
# contour geometry
# ---------------------------------------------------------------------------
def _trap(n):
    w = np.ones(n)
    if n > 1:
        w[0] = w[-1] = 0.5
    return w


def box_segments(lo, hi):
    """Edges (2-D, len(lo) == 2) or faces (3-D) of the node box [lo, hi].

    Returns a list of (coords (m, d) int, normal (3,), weights (m,))."""
    d = len(lo)
    segs = []
    for ax in range(d):
        others = [a for a in range(d) if a != ax]
        ranges = [np.arange(lo[a], hi[a] + 1) for a in others]
        grids = np.meshgrid(*ranges, indexing="ij")
        wts = _trap(ranges[0].size)
        if d == 3:
            wts = np.outer(_trap(ranges[0].size), _trap(ranges[1].size))
        for side, pos in ((-1, lo[ax]), (1, hi[ax])):
            coords = np.zeros(grids[0].shape + (d,), dtype=np.int64)
            for a, g in zip(others, grids):
                coords[..., a] = g
            coords[..., ax] = pos
            nrm = np.zeros(3)
            nrm[ax] = side
            segs.append((coords.reshape(-1, d), nrm, wts.reshape(-1)))
    return segs


def box_nodes(lo, hi):
    """Unique node coordinates of the box surface, sorted in linear-index
    order (x fastest); returns (coords (p, d))."""
    segs = box_segments(lo, hi)
    allc = np.concatenate([s[0] for s in segs])
    d = len(lo)
    key = allc[:, d - 1].copy()
    for a in range(d - 2, -1, -1):
        key = key * 100003 + allc[:, a]
    _, idx = np.unique(key, return_index=True)
    return allc[idx]


def linear_index(coords, n):
    """Linear cell index (x fastest) of integer coords for grid sizes n."""
    coords = np.asarray(coords)
    idx = np.zeros(coords.shape[0], dtype=np.int64)
    stride = 1
    for a in range(coords.shape[1]):
        idx += coords[:, a] * stride
        stride *= n[a]
    return idx


# ---------------------------------------------------------------------------
# radiation integrals
# ---------------------------------------------------------------------------
def _lookup(nodes, values):
    """Map from node coordinate tuple -> row of values."""
    return {tuple(c): v for c, v in zip(map(tuple, nodes), values)}


def radiation_vectors(nodes, Es, Hs, lo, hi, k, rhat, center):
    """N, L (complex, shape (n_dirs, 3)) for far-field directions rhat
    (n_dirs, 3) from scattered phasors Es, Hs (p, 3) at `nodes` (p, d)."""
    d = len(lo)
    tabE = _lookup(nodes, Es)
    tabH = _lookup(nodes, Hs)
    rhat = np.atleast_2d(rhat)
    N = np.zeros((rhat.shape[0], 3), complex)
    L = np.zeros((rhat.shape[0], 3), complex)
    for coords, nrm, w in box_segments(lo, hi):
        E = np.array([tabE[tuple(c)] for c in coords])
        H = np.array([tabH[tuple(c)] for c in coords])
        J = np.cross(nrm, H)          # J = n x H
        M = -np.cross(nrm, E)         # M = -n x E
        rp = np.zeros((coords.shape[0], 3))
        rp[:, :d] = coords - np.asarray(center)[:d]
        ph = np.exp(1j * k * (rhat @ rp.T)) * w[None, :]   # (dirs, nodes)
        N += ph @ J
        L += ph @ M
    return N, L


def farfield_2d(nodes, Es, Hs, lo, hi, k, theta_deg, pol, center, inc_amp):
    """|S(theta)|^2 (section 2.3, Eq. S2D) with theta measured in the xy
    plane from +x (callers add the incidence angle)."""
    th = np.deg2rad(np.asarray(theta_deg, dtype=float))
    rhat = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)
    N, L = radiation_vectors(nodes, Es, Hs, lo, hi, k, rhat, center)
    rxL = np.cross(rhat, L)
    rxN = np.cross(rhat, N)
    if pol == "TM":
        P = N[:, 2] - rxL[:, 2]
    else:
        P = L[:, 2] + rxN[:, 2]
    return k ** 2 / (8.0 * np.pi) * np.abs(P) ** 2 / abs(inc_amp) ** 2


def farfield_3d(nodes, Es, Hs, lo, hi, k, theta_deg, phi_deg, center, inc_amp):
    """|S(theta, phi)|^2 (section 2.3, Eq. S3D); theta from +z, phi from +x."""
    th = np.deg2rad(np.asarray(theta_deg, dtype=float))
    ph = np.deg2rad(np.broadcast_to(np.asarray(phi_deg, dtype=float), th.shape))
    st, ct, sp_, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    rhat = np.stack([st * cp, st * sp_, ct], axis=1)
    that = np.stack([ct * cp, ct * sp_, -st], axis=1)
    phat = np.stack([-sp_, cp, np.zeros_like(th)], axis=1)
    N, L = radiation_vectors(nodes, Es, Hs, lo, hi, k, rhat, center)
    Nt, Np = np.sum(N * that, 1), np.sum(N * phat, 1)
    Lt, Lp = np.sum(L * that, 1), np.sum(L * phat, 1)
    return (k ** 4 / (16 * np.pi ** 2) * (np.abs(Nt + Lp) ** 2 + np.abs(Np - Lt) ** 2)
            / abs(inc_amp) ** 2)


# ---------------------------------------------------------------------------
# closed-form radiators used to pin the transform
# ---------------------------------------------------------------------------
def dipole_fields(R, k):
    """Exact fields of a unit electric dipole along +x at the origin,
    exp(+j omega t) convention, unit impedance (c = 1 after rescaling time):
      E = 1/(4pi) {k^2 (n x p) x n e^{-jkr}/r + [3n(n.p) - p](1/r^3 + jk/r^2) e^{-jkr}}
      H = k^2/(4pi) (n x p) (e^{-jkr}/r) (1 + 1/(jkr)).
    Far-field intensity: k^2 r^2 |E|^2 = k^6 sin^2(gamma)/(16 pi^2)."""
    r = np.linalg.norm(R, axis=-1, keepdims=True)
    n = R / r
    p = np.array([1.0, 0, 0])
    e = np.exp(-1j * k * r)
    nxp = np.cross(n, p)
    E = (k ** 2 * np.cross(nxp, n) * e / r
         + (3 * n * np.sum(n * p, -1, keepdims=True) - p) * (1 / r ** 3 + 1j * k / r ** 2) * e) / (4 * np.pi)
    H = k ** 2 / (4 * np.pi) * nxp * e / r * (1 + 1 / (1j * k * r))
    return E, H


def farfield_2d_amplitude(nodes, Es, Hs, lo, hi, k, theta_deg, pol, center):
    """Complex far-field combination P(theta) with |S|^2 = k^2/(8 pi) |P|^2
    / |E_i|^2: P = N_z - (rhat x L)_z (TM) or L_z + (rhat x N)_z (TE).
    Linear in the phasors (used by the adjoint objective)."""
    th = np.deg2rad(np.asarray(theta_deg, dtype=float))
    rhat = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)
    N, L = radiation_vectors(nodes, Es, Hs, lo, hi, k, rhat, center)
    if pol == "TM":
        return N[:, 2] - np.cross(rhat, L)[:, 2]
    return L[:, 2] + np.cross(rhat, N)[:, 2]
