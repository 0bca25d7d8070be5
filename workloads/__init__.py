"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds only input construction -- permittivity maps (staircase
rasterisation of the paper's scatterers), plane-wave parameters, contour
boxes, DFT windows and the seeded batch / design-region recipes.  It
contains none of the lattice Boltzmann arithmetic, so that the oracle and
the HIP library can both consume its outputs while sharing no method code.

Geometry reading (the paper does not state its sub-cell treatment; its
interfaces are sharp, section 3.1): a cell takes the inside permittivity
when its centre lies strictly inside the shape.  Scatterers are centred at
((n - 1)/2, ...).  The hexagon has circumradius a (section 3.3) with a
vertex on +x.
"""
from dataclasses import dataclass, field

import numpy as np

SIGMA_MAX = 0.25          # absorbing-layer strength (reading, fixed once)
RAMP_PERIODS = 3.0        # source ramp length in periods


# ---------------------------------------------------------------------------
# permittivity maps, arrays indexed [z][y][x]
# ---------------------------------------------------------------------------
def half_space(nx, ny, x0, eps_in, nz=1):
    """eps_in for x >= x0, 1 elsewhere (planar interface, section 3.1)."""
    e = np.ones((nz, ny, nx))
    e[:, :, x0:] = eps_in
    return e


def circle(n, a, eps_in, center=None, ny=None):
    ny = n if ny is None else ny
    cx, cy = ((n - 1) / 2.0, (ny - 1) / 2.0) if center is None else center
    y, x = np.mgrid[0:ny, 0:n]
    e = np.ones((1, ny, n))
    e[0][(x - cx) ** 2 + (y - cy) ** 2 < a * a] = eps_in
    return e


def hexagon(n, a, eps_in, center=None, ny=None):
    """Regular hexagon of circumradius a, one vertex on +x."""
    ny = n if ny is None else ny
    cx, cy = ((n - 1) / 2.0, (ny - 1) / 2.0) if center is None else center
    y, x = np.mgrid[0:ny, 0:n]
    X, Y = np.abs(x - cx), np.abs(y - cy)
    apo = a * np.sqrt(3.0) / 2.0          # apothem
    inside = (Y < apo) & (np.sqrt(3.0) * X + Y < np.sqrt(3.0) * a)
    e = np.ones((1, ny, n))
    e[0][inside] = eps_in
    return e


def sphere(n, a, eps_in):
    c = (n - 1) / 2.0
    z, y, x = np.ogrid[0:n, 0:n, 0:n]
    r2 = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
    e = np.ones((n, n, n), dtype=np.float64)
    e[r2 < a * a] = eps_in
    return e


# ---------------------------------------------------------------------------
# plane waves and contours
# ---------------------------------------------------------------------------
def plane_wave_2d(theta_deg, pol):
    """(khat, ehat) for a 2-D run: propagation in the xy plane at angle theta
    from +x.  TM: E along z (the cylinder axis); TE: E in-plane with
    H = khat x E along +z."""
    th = np.deg2rad(theta_deg)
    k = np.array([np.cos(th), np.sin(th), 0.0])
    if pol == "TM":
        e = np.array([0.0, 0.0, 1.0])
    elif pol == "TE":
        e = np.array([-np.sin(th), np.cos(th), 0.0])   # zhat x khat
    else:
        raise ValueError(pol)
    return k, e


def box_around_center(n, half):
    """Node box [lo, hi] symmetric about the grid centre (n - 1)/2; `half`
    is the half-width in cells and must make lo an integer."""
    lo = tuple(int(round((m - 1) / 2.0 - half)) for m in n)
    hi = tuple(int(round((m - 1) / 2.0 + half)) for m in n)
    return lo, hi


def period_steps(lam):
    """Steps per source period, T = 3 lambda (omega = 2 pi/(3 lambda))."""
    T = 3.0 * lam
    if abs(T - round(T)) > 1e-9:
        raise ValueError("lambda must make 3*lambda an integer")
    return int(round(T))


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------
@dataclass
class Case2D:
    name: str
    nx: int
    ny: int
    eps: np.ndarray
    lam: float
    theta_deg: float
    pol: str
    absorb: tuple
    steps: int
    box_lo: tuple = None
    box_hi: tuple = None
    radius: float = 0.0
    eps_in: float = 1.0
    shape: str = "circle"
    extra: dict = field(default_factory=dict)

    @property
    def window(self):
        T = period_steps(self.lam)
        return self.steps - T, T


def fresnel_case(theta_deg=0.0, pol="TM", nx=256, ny=None, steps=3000, eps_in=2.25, lam=32.0):
    """Planar interface: eps_in for x >= nx/2, absorbing x faces (W = 20), y
    periodic.  At 30 degrees and lambda = 32, k_y = k/2 repeats every 64
    cells, so ny = 64 (or 128) is exactly periodic."""
    if ny is None:
        ny = 1 if theta_deg == 0 else 64
    eps = half_space(nx, ny, nx // 2, eps_in)
    return Case2D("fresnel", nx, ny, eps, lam, theta_deg, pol, (20, 0, 0), steps, eps_in=eps_in,
                  shape="half-space")


def planar_sweep_case(eps_in, mu_in, pol="TM", lam_wall=20.0, W=20):
    """One point of the section 3.1 material sweep: normal incidence from
    vacuum onto a half space (eps_in, mu_in) on a single-row grid, resolved
    with lam_wall = lambda / sqrt(eps mu) cells inside the medium (lambda
    rounded so that 3 lambda is integral).  The vacuum side holds 1.5 free-
    space wavelengths, the medium 5 inner wavelengths (+16 cells each), and
    the run lasts the ramp plus two vacuum crossings and two medium
    crossings plus one period, so the DFT window sees the steady state.
    case.extra holds the interface column x0 and the permeability map mu."""
    n = float(np.sqrt(eps_in * mu_in))
    lam = round(3.0 * lam_wall * n) / 3.0
    Lv = int(1.5 * lam) + 16
    Lm = int(5.0 * lam / n) + 16
    nx = W + Lv + Lm + W
    x0 = W + Lv
    T = period_steps(lam)
    steps = int(9.0 * lam + 6 * (Lv + W) + 6 * n * (Lm + W)) + T
    eps = half_space(nx, 1, x0, eps_in)
    mu = half_space(nx, 1, x0, mu_in)
    return Case2D(f"sweep-eps{eps_in:g}-mu{mu_in:g}", nx, 1, eps, lam, 0.0, pol, (W, 0, 0), steps,
                  eps_in=eps_in, shape="half-space", extra={"x0": x0, "mu": mu, "mu_in": mu_in})


def cylinder_case(eps_in=2.25, pol="TM", n=1024, a=25.5, lam=32.0, W=32, steps=8000,
                  half=34.5, theta_deg=0.0, shape="circle"):
    """Infinite dielectric cylinder (x = 2 pi a / lambda = 5.007 at a = 25.5,
    lambda = 32), centred, absorbing on all four faces."""
    if shape == "circle":
        eps = circle(n, a, eps_in)
    else:
        eps = hexagon(n, a, eps_in)
    lo, hi = box_around_center((n, n), half)
    return Case2D("cylinder", n, n, eps, lam, theta_deg, pol, (W, W, 0), steps, lo, hi, a, eps_in,
                  shape)


def vacuum_companion(case):
    """Same grid, layers, source and window, eps = 1 everywhere."""
    c = Case2D(case.name + "-vacuum", case.nx, case.ny, np.ones_like(case.eps), case.lam,
               case.theta_deg, case.pol, case.absorb, case.steps, case.box_lo, case.box_hi,
               case.radius, 1.0, case.shape)
    return c


def batch_cases(count=64, seed=251011042, W=32, steps=6000, stress=False):
    """Seeded batch of uneven 2-D scatterers: shape circle/hexagon (p = 1/2),
    eps_r ~ U[1.5, 4], size parameter x ~ U[1, 10], lambda ~ U{24..40},
    incidence ~ U[0, 60] degrees, TM.  Side = roundup64(max(256, 6 lambda +
    2a + 2W)); with stress=True the side is drawn from {256, 320, ..., 1536}
    instead (the stated 256..1536 range)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        shape = "circle" if rng.random() < 0.5 else "hexagon"
        eps_in = rng.uniform(1.5, 4.0)
        x = rng.uniform(1.0, 10.0)
        lam = float(rng.integers(24, 41))
        theta = rng.uniform(0.0, 60.0)
        a = x * lam / (2 * np.pi)
        side = int(np.ceil(max(256.0, 6 * lam + 2 * a + 2 * W) / 64.0) * 64)
        if stress:
            side = int(rng.integers(4, 25)) * 64
        half = np.ceil(a) + max(6, int(np.ceil(lam / 4))) + 0.5
        if half > (side - 1) / 2.0 - W - 4:
            half = np.floor((side - 1) / 2.0 - W - 4) + 0.5
        c = cylinder_case(eps_in, "TM", side, a, lam, W, steps, half, theta, shape)
        c.name = f"batch{i}"
        out.append(c)
    return out


def design_region(n=1024, size=128, seed=11042, lo=1.0, hi=4.0):
    """Centred size x size design region with eps ~ U[lo, hi]; returns the
    full eps map and the region's (x0, y0)."""
    rng = np.random.default_rng(seed)
    eps = np.ones((1, n, n))
    x0 = (n - size) // 2
    eps[0, x0:x0 + size, x0:x0 + size] = rng.uniform(lo, hi, (size, size))
    return eps, (x0, x0)


@dataclass
class Case3D:
    n: int
    eps: np.ndarray
    lam: float
    W: int
    steps: int
    box_lo: tuple
    box_hi: tuple
    radius: float
    eps_in: float

    @property
    def window(self):
        T = period_steps(self.lam)
        return self.steps - T, T


def sphere_case(n=384, x_size=6.0, lam=24.0, eps_in=2.25, W=24, steps=4000, half=29.5,
                with_eps=True):
    a = x_size * lam / (2 * np.pi)
    eps = sphere(n, a, eps_in) if with_eps else None
    lo, hi = box_around_center((n, n, n), half)
    return Case3D(n, eps, lam, W, steps, lo, hi, a, eps_in)
