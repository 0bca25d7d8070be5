"""Inverse-design objective and its discrete-adjoint gradient on the oracle.

TEST INFRASTRUCTURE ONLY.

Objective (inverse design of the far field, TM, 2-D):
    J(eps) = sum_theta w_theta |S(theta)|^2,
with |S|^2 from the near-to-far-field transform of section 2.4 applied to
the scattered phasors (total run minus the eps = 1 companion run, which does
not depend on eps) and normalised by the companion's incident amplitude.
The phasors are X = (2/(M T)) sum_t F(t) exp(-j omega t), so
    dJ/dF_q(t) = sum_theta w_theta kappa 2 Re(conj(P_theta) A_theta,q (2/(MT)) e^{-j omega t}),
kappa = k^2/(8 pi |E_i|^2), with P_theta = A_theta . X_scattered the complex
far-field combination (linear in X; A is read off column by column).
The gradient dJ/deps then comes from the oracle's reverse sweep
(lbm_oracle.c: oracle_adjoint) over the stored forward states.
"""
import numpy as np

from . import ntff
from .core import Oracle
from .run import probe_node


def _amplitude_matrix(case, nodes, k, theta_abs):
    """A[theta, node*6 + comp] so that P = A @ X.ravel()."""
    center = ((case.nx - 1) / 2.0, (case.ny - 1) / 2.0)
    p = len(nodes)
    A = np.zeros((len(theta_abs), p * 6), complex)
    for q in range(p * 6):
        X = np.zeros((p, 6), complex)
        X.flat[q] = 1.0
        A[:, q] = ntff.farfield_2d_amplitude(nodes, X[:, :3], X[:, 3:], case.box_lo, case.box_hi, k,
                                             theta_abs, case.pol, center)
    return A


def _run(case, eps, sigma_max, ramp_periods, keep_history):
    from workloads import plane_wave_2d

    o = Oracle(case.nx, case.ny, 1, case.absorb, sigma_max)
    o.set_eps(eps)
    kh, eh = plane_wave_2d(case.theta_deg, case.pol)
    o.set_source(case.lam, kh, eh, 1.0, ramp_periods)
    nodes = ntff.box_nodes(case.box_lo, case.box_hi)
    cells = ntff.linear_index(nodes, (case.nx, case.ny))
    pr = ntff.linear_index(np.array([probe_node(case.box_lo, case.box_hi)]), (case.nx, case.ny))
    w0, wl = case.window
    o.set_dft(np.concatenate([cells, pr]), w0, wl)
    hist = None
    if keep_history:
        hist = np.empty((case.steps,) + o.shape + (7, 6))
        for t in range(case.steps):
            hist[t] = o.get_state()
            o.step(1)
    else:
        o.step(case.steps)
    X = o.get_dft()
    return o, nodes, cells, X[:-1], X[-1], hist


class FarFieldObjective:
    """J(eps) = sum_theta w_theta |S(theta)|^2 for a workloads.Case2D."""

    def __init__(self, case, theta_rel_deg, weights=None, sigma_max=0.25, ramp_periods=3.0):
        self.case = case
        self.theta = np.asarray(theta_rel_deg, dtype=float)
        self.w = np.ones_like(self.theta) if weights is None else np.asarray(weights, float)
        self.sigma_max, self.ramp = sigma_max, ramp_periods
        self.k = 2 * np.pi / case.lam
        from workloads import vacuum_companion

        _, self.nodes, self.cells, Xi, pi_, _ = _run(vacuum_companion(case), np.ones_like(case.eps),
                                                      sigma_max, ramp_periods, False)
        self.X_inc = Xi
        self.inc_amp = pi_[2] if case.pol == "TM" else pi_[5]
        self.A = _amplitude_matrix(case, self.nodes, self.k, self.theta + case.theta_deg)
        self.kappa = self.k ** 2 / (8 * np.pi * abs(self.inc_amp) ** 2)

    def value(self, eps):
        _, _, _, X, _, _ = _run(self.case, eps, self.sigma_max, self.ramp, False)
        P = self.A @ (X - self.X_inc).ravel()
        return float(np.sum(self.w * self.kappa * np.abs(P) ** 2))

    def value_and_gradient(self, eps):
        c = self.case
        o, _, cells, X, _, hist = _run(c, eps, self.sigma_max, self.ramp, True)
        P = self.A @ (X - self.X_inc).ravel()
        J = float(np.sum(self.w * self.kappa * np.abs(P) ** 2))
        # dJ/dX (as the coefficient g with dJ = 2 Re(g . dX))
        g = (self.w * self.kappa * np.conj(P)) @ self.A          # (p*6,)
        g = g.reshape(-1, 6)
        w0, wl = c.window
        omega = 2 * np.pi / (3 * c.lam)
        dJdF = np.zeros((c.steps, o.ncell, 6))
        for t in range(w0, w0 + wl):
            ph = (2.0 / wl) * np.exp(-1j * omega * t)
            dJdF[t, cells, :] = 2.0 * np.real(g * ph)
        grad = o.adjoint(hist, dJdF, 0)
        return J, grad
