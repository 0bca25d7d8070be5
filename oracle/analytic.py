"""Closed forms the oracle is pinned against (FP64).

TEST INFRASTRUCTURE ONLY.

- Fresnel amplitude coefficients at a planar interface (section 3.1,
  Eq. ref_trans gives normal incidence; the oblique s/p forms are the
  textbook generalisation, needed for 30 degree incidence).
- Lattice dispersion of the D3Q7 scheme (section 2.1).  The recovered
  Maxwell equations have c = 1/3 and second-order error; the exact
  dispersion of the discrete scheme for a wave along a lattice axis is
  derived here from Eq. LBGK_equation and Eq. EDF in Fourier space:

  Vacuum, wave along +x, fields (E_z, H_y).  With a = e_{+x,z},
  u = (sum of the four transverse e_z) - (their h_y), one step reads
      a(x+1, t+1) = (u - a)/3,     u(x, t+1) = (8 a + u)/3.
  With a, u ~ exp(i(kx - omega t)) this gives
      3 w Z^2 + (1 - w) Z - 3 = 0,  w = e^{ik}, Z = e^{-i omega},
  i.e.  sin(k/2 - omega) = sin(k/2) / 3.

  Uniform dielectric (eps_r): the rest population e_0 and the left-moving
  populations couple in; dispersion_axis() solves the 2x2 Fourier symbol
  in (E_z, H_y) for arbitrary eps_r numerically.
"""
import numpy as np
from scipy.optimize import brentq


# ---------------------------------------------------------------------------
# Fresnel
# ---------------------------------------------------------------------------
def fresnel_normal(eps_r, mu_r=1.0):
    """Reflected / transmitted E amplitude ratios at normal incidence from
    vacuum onto (eps_r, mu_r) -- section 3.1, Eq. ref_trans."""
    sm, se = np.sqrt(mu_r), np.sqrt(eps_r)
    return (sm - se) / (sm + se), 2.0 * sm / (sm + se)


def fresnel_oblique(eps_r, theta_i_deg, pol):
    """Textbook Fresnel E-amplitude coefficients from vacuum onto a
    non-magnetic medium n = sqrt(eps_r).

    pol='s': E perpendicular to the plane of incidence (for a 2-D run with
    the interface normal in-plane this is TM_z, E along the invariant axis);
    pol='p': E in the plane of incidence (TE_z).  Returns (r, t, theta_t)."""
    n = np.sqrt(eps_r)
    ti = np.deg2rad(theta_i_deg)
    tt = np.arcsin(np.sin(ti) / n)
    ci, ct = np.cos(ti), np.cos(tt)
    if pol == "s":
        r = (ci - n * ct) / (ci + n * ct)
        t = 2 * ci / (ci + n * ct)
    elif pol == "p":
        r = (n * ci - ct) / (n * ci + ct)
        t = 2 * ci / (n * ci + ct)
    else:
        raise ValueError(pol)
    return r, t, tt


# ---------------------------------------------------------------------------
# Lattice dispersion
# ---------------------------------------------------------------------------
def omega_vacuum_axis(k):
    """Physical branch of sin(k/2 - omega) = sin(k/2)/3 (see module doc)."""
    k = np.asarray(k, dtype=float)
    return k / 2.0 - np.arcsin(np.sin(k / 2.0) / 3.0)


def k_vacuum_axis(omega):
    """Inverse of omega_vacuum_axis on 0 < k < pi."""
    return brentq(lambda k: omega_vacuum_axis(k) - omega, 1e-12, np.pi - 1e-12, xtol=1e-15)


def _poly(*factors):
    """Product of polynomials in Z given as coefficient lists (lowest first)."""
    out = np.array([1.0 + 0j])
    for f in factors:
        out = np.polynomial.polynomial.polymul(out, np.asarray(f, dtype=complex))
    return out


def dispersion_axis(k, eps=1.0):
    """omega(k) of the physical (forward, low-frequency) branch for a TM wave
    along a lattice axis in a uniform medium eps_r (mu_r = 1).

    Fourier symbol (see module doc), with w = e^{ik}, Z = e^{-i omega} and
    the one-step factors  a = (E - H)/(3 (wZ + 1)),  b = (E + H)/(3 (Z/w + 1)),
    s_e = 4E/(3 (Z + 1)),  s_h = 4H/(3 (Z + 1)),  e_0 = 2 (eps - 1) E/(Z + 1):
        eps E = a + b + s_e + e_0,      H = -a + b + s_h.
    Clearing the denominators P = (wZ+1)(Z/w+1)(Z+1) gives a degree-6
    polynomial whose unit-circle root nearest the continuum value is taken.
    """
    w = np.exp(1j * k)
    A = [1.0, w]            # wZ + 1
    B = [1.0, 1.0 / w]      # Z/w + 1
    G = [1.0, 1.0]          # Z + 1
    P = _poly(A, B, G)
    pad = lambda c: np.pad(c, (0, 4 - len(c)))
    m11 = pad(_poly(B, G) / 3 + _poly(A, G) / 3 + _poly(A, B) * (4.0 / 3 + 2 * (eps - 1))) - eps * P
    m22 = pad(_poly(B, G) / 3 + _poly(A, G) / 3 + _poly(A, B) * (4.0 / 3)) - P
    m12 = pad(-_poly(B, G) / 3 + _poly(A, G) / 3)
    det = np.polynomial.polynomial.polysub(np.polynomial.polynomial.polymul(m11, m22),
                                           np.polynomial.polynomial.polymul(m12, m12))
    roots = np.polynomial.polynomial.polyroots(det)
    roots = roots[np.abs(np.abs(roots) - 1.0) < 1e-8]
    om = -np.angle(roots)
    guess = k / (3.0 * np.sqrt(eps))
    return float(om[np.argmin(np.abs(om - guess))])
