"""Lorenz-Mie references (FP64), written from the textbook series.

TEST INFRASTRUCTURE ONLY.

The paper compares its LBM far fields with Lorenz-Mie theory for infinite
circular cylinders (section 3.2) and spheres (section 3.4) without printing
the series; the standard forms of Bohren & Huffman, "Absorption and
Scattering of Light by Small Particles" (ch. 4 and 8) are used here:

Cylinder, normal incidence, relative index m, size parameter x = k a:
  b_n = [J_n(mx) J_n'(x) - m J_n'(mx) J_n(x)] / [J_n(mx) H_n'(x) - m J_n'(mx) H_n(x)]
  a_n = [m J_n(mx) J_n'(x) - J_n(x) J_n'(mx)] / [m J_n(mx) H_n'(x) - J_n'(mx) H_n(x)]
  T1(theta) = b_0 + 2 sum b_n cos(n theta)   (E parallel to the axis = TM here)
  T2(theta) = a_0 + 2 sum a_n cos(n theta)   (E perpendicular      = TE here)
  PEC (m -> infinity): b_n = J_n(x)/H_n(x), a_n = J_n'(x)/H_n'(x).
Sphere:
  a_n = [m psi_n(mx) psi_n'(x) - psi_n(x) psi_n'(mx)] / [m psi_n(mx) xi_n'(x) - xi_n(x) psi_n'(mx)]
  b_n = [psi_n(mx) psi_n'(x) - m psi_n(x) psi_n'(mx)] / [psi_n(mx) xi_n'(x) - m xi_n(x) psi_n'(mx)]
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),  S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n)

Near fields (used to pin the near-to-far-field transform of section 2.4):
  cylinder_near_field -- the scattered z-field series with its curl;
  sphere_near_field   -- the scattered field in vector spherical harmonics
                         (section 4.4 of the book).

Intensities in the paper's normalisation (section 2.3, Eq. S2D / S3D):
  2-D  |S(theta)|^2 = k r |E_s|^2/|E_i|^2 = (2/pi) |T(theta)|^2
  3-D  |S(theta,phi)|^2 = k^2 r^2 |E_s|^2/|E_i|^2 = |S2|^2 cos^2 phi + |S1|^2 sin^2 phi,
       phi measured from the incident E direction.
"""
import numpy as np
from scipy import special as sp


def _nmax(x):
    return int(np.ceil(abs(x) + 4.0 * abs(x) ** (1.0 / 3.0) + 2.0)) + 4


# ---------------------------------------------------------------------------
# circular cylinder
# ---------------------------------------------------------------------------
def cylinder_coefficients(x, m, nmax=None):
    """(a_n, b_n) for n = 0..nmax; m = None means a perfect conductor."""
    if nmax is None:
        nmax = _nmax(x)
    n = np.arange(nmax + 1)
    Jx, dJx = sp.jv(n, x), sp.jvp(n, x)
    Hx, dHx = sp.hankel1(n, x), sp.h1vp(n, x)
    if m is None:
        return dJx / dHx, Jx / Hx
    Jm, dJm = sp.jv(n, m * x), sp.jvp(n, m * x)
    a = (m * Jm * dJx - Jx * dJm) / (m * Jm * dHx - dJm * Hx)
    b = (Jm * dJx - m * dJm * Jx) / (Jm * dHx - m * dJm * Hx)
    return a, b


def cylinder_T(theta_deg, x, m, pol):
    """Amplitude T1 (pol='TM', E along the axis) or T2 (pol='TE')."""
    a, b = cylinder_coefficients(x, m)
    c = b if pol == "TM" else a
    th = np.deg2rad(np.asarray(theta_deg, dtype=float))
    n = np.arange(1, c.size)
    return c[0] + 2.0 * np.cos(np.outer(th, n)) @ c[1:]


def cylinder_S2(theta_deg, x, m, pol):
    """|S(theta)|^2 in the paper's 2-D normalisation: (2/pi)|T|^2."""
    return (2.0 / np.pi) * np.abs(cylinder_T(theta_deg, x, m, pol)) ** 2


def cylinder_efficiencies(x, m, pol):
    """(Q_ext, Q_sca) per unit length, normalised by the diameter."""
    a, b = cylinder_coefficients(x, m)
    c = b if pol == "TM" else a
    qsca = (2.0 / x) * (abs(c[0]) ** 2 + 2.0 * np.sum(np.abs(c[1:]) ** 2))
    qext = (2.0 / x) * np.real(c[0] + 2.0 * np.sum(c[1:]))
    return qext, qsca


def cylinder_near_field(X, Y, x_size, k, m, pol):
    """Scattered field of a unit incident plane wave exp(i k x) (time factor
    exp(-i omega t)) around a cylinder of size parameter x_size = k a centred
    at the origin, outside it.  Returns (E, H) complex arrays (..., 3) in
    units with unit wave impedance (H = curl E / (i k)).

    TM (E along z):  E_z^s = -sum_n i^n b_n H_n(kr) e^{i n phi}
    TE (H along z):  H_z^s = -sum_n i^n a_n H_n(kr) e^{i n phi}
    (the PEC limits reproduce E_z = 0 resp. dH_z/dr = 0 on the surface).
    """
    a, b = cylinder_coefficients(x_size, m)
    c = b if pol == "TM" else a
    N = c.size - 1
    r = np.hypot(X, Y)
    ph = np.arctan2(Y, X)
    kr = k * r
    F = np.zeros(r.shape, complex)
    dF_dr = np.zeros(r.shape, complex)
    dF_dph = np.zeros(r.shape, complex)
    for n in range(-N, N + 1):
        cn = c[abs(n)] * (1j ** n) * np.exp(1j * n * ph)
        Hn = sp.hankel1(n, kr)
        dHn = sp.h1vp(n, kr)
        F += -cn * Hn
        dF_dr += -cn * k * dHn
        dF_dph += -cn * 1j * n * Hn
    E = np.zeros(r.shape + (3,), complex)
    H = np.zeros(r.shape + (3,), complex)
    # curl(z F) = r_hat (1/r) dF/dphi - phi_hat dF/dr
    cr = dF_dph / r
    cp = -dF_dr
    cx = cr * np.cos(ph) - cp * np.sin(ph)
    cy = cr * np.sin(ph) + cp * np.cos(ph)
    if pol == "TM":
        E[..., 2] = F
        H[..., 0] = cx / (1j * k)        # H = curl E / (i k)
        H[..., 1] = cy / (1j * k)
    else:
        H[..., 2] = F
        E[..., 0] = -cx / (1j * k)       # E = -curl H / (i k)
        E[..., 1] = -cy / (1j * k)
    return E, H


# ---------------------------------------------------------------------------
# sphere
# ---------------------------------------------------------------------------
def _riccati(n, z):
    """psi_n(z) = z j_n(z), psi_n'(z), xi_n(z) = z h_n^(1)(z), xi_n'(z)."""
    j, dj = sp.spherical_jn(n, z), sp.spherical_jn(n, z, derivative=True)
    psi, dpsi = z * j, j + z * dj
    y, dy = sp.spherical_yn(n, z), sp.spherical_yn(n, z, derivative=True)
    xi = z * (j + 1j * y)
    dxi = (j + 1j * y) + z * (dj + 1j * dy)
    return psi, dpsi, xi, dxi


def sphere_coefficients(x, m, nmax=None):
    if nmax is None:
        nmax = _nmax(x)
    n = np.arange(1, nmax + 1)
    px, dpx, xx, dxx = _riccati(n, x)
    pm, dpm, _, _ = _riccati(n, m * x)
    a = (m * pm * dpx - px * dpm) / (m * pm * dxx - xx * dpm)
    b = (pm * dpx - m * px * dpm) / (pm * dxx - m * xx * dpm)
    return a, b


def sphere_S1S2(theta_deg, x, m):
    a, b = sphere_coefficients(x, m)
    N = a.size
    mu = np.cos(np.deg2rad(np.asarray(theta_deg, dtype=float)))
    pi_prev = np.zeros_like(mu)          # pi_0
    pi_cur = np.ones_like(mu)            # pi_1
    S1 = np.zeros(mu.shape, complex)
    S2 = np.zeros(mu.shape, complex)
    for n in range(1, N + 1):
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (a[n - 1] * pi_cur + b[n - 1] * tau)
        S2 += f * (a[n - 1] * tau + b[n - 1] * pi_cur)
        pi_next = ((2 * n + 1) / n) * mu * pi_cur - ((n + 1) / n) * pi_prev
        pi_prev, pi_cur = pi_cur, pi_next
    return S1, S2


def sphere_S2(theta_deg, phi_deg, x, m):
    """|S(theta, phi)|^2 = |S2|^2 cos^2 phi + |S1|^2 sin^2 phi."""
    S1, S2 = sphere_S1S2(theta_deg, x, m)
    ph = np.deg2rad(phi_deg)
    return np.abs(S2) ** 2 * np.cos(ph) ** 2 + np.abs(S1) ** 2 * np.sin(ph) ** 2


def sphere_near_field(R, x_size, k, m):
    """Scattered field of a unit incident plane wave x_hat exp(i k z) (time
    factor exp(-i omega t)) around a sphere of size parameter x_size = k a
    centred at the origin, at points R (..., 3) outside it; units with unit
    wave impedance.  Bohren & Huffman, section 4.4:
        E_s = sum_n E_n (i a_n N_e1n - b_n M_o1n),
        H_s = sum_n E_n (i b_n N_o1n + a_n M_e1n),   E_n = i^n (2n+1)/(n(n+1)),
    with the vector spherical harmonics of the outgoing spherical Hankel
    function h_n^(1)(kr):
        M_o1n = cos(phi) pi_n h_n e_theta - sin(phi) tau_n h_n e_phi
        M_e1n = -sin(phi) pi_n h_n e_theta - cos(phi) tau_n h_n e_phi
        N_o1n = sin(phi) n(n+1) sin(theta) pi_n h_n/rho e_r
                + sin(phi) tau_n D_n e_theta + cos(phi) pi_n D_n e_phi
        N_e1n = cos(phi) n(n+1) sin(theta) pi_n h_n/rho e_r
                + cos(phi) tau_n D_n e_theta - sin(phi) pi_n D_n e_phi
    where rho = kr and D_n = (rho h_n)'/rho.  Returns (E, H), (..., 3)."""
    a, b = sphere_coefficients(x_size, m)
    R = np.asarray(R, dtype=float)
    r = np.linalg.norm(R, axis=-1)
    th = np.arccos(np.clip(R[..., 2] / r, -1.0, 1.0))
    ph = np.arctan2(R[..., 1], R[..., 0])
    rho = k * r
    mu, st = np.cos(th), np.sin(th)
    cp, sp_ = np.cos(ph), np.sin(ph)
    Er = np.zeros(r.shape, complex)
    Et = np.zeros(r.shape, complex)
    Ep = np.zeros(r.shape, complex)
    Hr = np.zeros(r.shape, complex)
    Ht = np.zeros(r.shape, complex)
    Hp = np.zeros(r.shape, complex)
    pi_prev, pi_cur = np.zeros_like(mu), np.ones_like(mu)
    for n in range(1, a.size + 1):
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        j, dj = sp.spherical_jn(n, rho), sp.spherical_jn(n, rho, derivative=True)
        y, dy = sp.spherical_yn(n, rho), sp.spherical_yn(n, rho, derivative=True)
        h, dh = j + 1j * y, dj + 1j * dy
        D = (h + rho * dh) / rho
        En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
        an, bn = a[n - 1], b[n - 1]
        radial = n * (n + 1) * st * pi_cur * h / rho
        # E: i a_n N_e1n - b_n M_o1n
        Er += En * (1j * an * cp * radial)
        Et += En * (1j * an * cp * tau * D - bn * cp * pi_cur * h)
        Ep += En * (-1j * an * sp_ * pi_cur * D + bn * sp_ * tau * h)
        # H: i b_n N_o1n + a_n M_e1n
        Hr += En * (1j * bn * sp_ * radial)
        Ht += En * (1j * bn * sp_ * tau * D - an * sp_ * pi_cur * h)
        Hp += En * (1j * bn * cp * pi_cur * D - an * cp * tau * h)
        pi_next = ((2 * n + 1) / n) * mu * pi_cur - ((n + 1) / n) * pi_prev
        pi_prev, pi_cur = pi_cur, pi_next

    def cart(Fr, Ft, Fp):
        out = np.zeros(r.shape + (3,), complex)
        out[..., 0] = Fr * st * cp + Ft * mu * cp - Fp * sp_
        out[..., 1] = Fr * st * sp_ + Ft * mu * sp_ + Fp * cp
        out[..., 2] = Fr * mu - Ft * st
        return out

    return cart(Er, Et, Ep), cart(Hr, Ht, Hp)


def sphere_efficiencies(x, m):
    a, b = sphere_coefficients(x, m)
    n = np.arange(1, a.size + 1)
    qext = (2.0 / x ** 2) * np.sum((2 * n + 1) * np.real(a + b))
    qsca = (2.0 / x ** 2) * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return qext, qsca
