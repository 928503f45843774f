"""Geometry, units, radial grid and Fourier wavenumbers (oracle side).

Readings taken where the paper is silent or ambiguous:

* Units (Sec. 2, Fig. 1): Re is defined with the inner-wall speed W_i and the
  full gap R_o - R_i, while the Appendix writes 1/Re in front of the viscous
  terms.  Lengths are therefore measured in units of the gap d (``gap``
  scales them), velocities in units of W_i, and nu = gap / Re.  Then
  R_i = gap * zeta / (1 - zeta) and R_o = gap / (1 - zeta).
* Radial grid (Sec. 2.1 says only "smoothly stretched"): N_r points including
  both walls, r_n = R_i + d (1 + T(xi_n)) / 2 with xi_n = -1 + 2 n / (N_r - 1)
  and T(xi) = tanh(s xi) / tanh(s), or T(xi) = xi when s = 0.
* Fourier domain (Sec. 4): the default azimuthal period is the paper's
  L_theta = 10 pi h measured at mid-gap, i.e. Theta = min(2 pi, 5 pi d / r_c)
  with r_c = (R_i + R_o) / 2, and the default axial period is L_z = 5 h =
  2.5 d.  Azimuthal wavenumbers m_j = 2 pi j / Theta need not be integers.
* Dealiasing (the paper does not state its rule): with N physical points the
  retained wavenumbers are |k| <= K = floor((N - 1) / 3), the exact 3/2 rule
  for quadratic products.  Only j >= 0 is stored; l runs over -K_z..K_z and is
  stored at index l + K_z.
"""

from dataclasses import dataclass, field

import math

import numpy as np


@dataclass
class Geometry:
    """Problem statement of one Taylor--Couette instance (Sec. 2, Fig. 1).

    ``re_outer`` is W_o d / nu of the outer wall (0 = at rest, the paper's
    standard set-up; Sec. 3 uses a counter-rotating outer wall once).
    ``theta_period`` and ``lz`` of 0 select the defaults of Sec. 4.
    ``stretch`` is the tanh parameter s of the radial grid (0 = uniform).
    """

    zeta: float
    re: float
    nr: int
    ntheta: int
    nz: int
    dt: float
    gap: float = 1.0
    re_outer: float = 0.0
    theta_period: float = 0.0
    lz: float = 0.0
    stretch: float = 0.0

    def validate(self):
        if not (0.0 < self.zeta < 1.0):
            raise ValueError("radius ratio must lie in (0, 1)")
        if not (self.gap > 0 and self.re > 0 and self.dt > 0):
            raise ValueError("gap, Re and dt must be positive")
        if self.nr < 7:
            raise ValueError("need at least 7 radial points")
        if self.ntheta < 4 or self.nz < 4:
            raise ValueError("need at least 4 points in theta and z")
        if self.stretch < 0:
            raise ValueError("stretch must be >= 0")


def truncation(n):
    """Largest retained wavenumber index for n physical points (3/2 rule)."""
    return (n - 1) // 3


@dataclass
class Discretisation:
    """Everything the oracle derives from a Geometry: radii, nu, grid,
    Fourier periods and wavenumbers."""

    geo: Geometry
    ri: float = field(init=False)
    ro: float = field(init=False)
    nu: float = field(init=False)
    r: np.ndarray = field(init=False)
    theta_period: float = field(init=False)
    lz: float = field(init=False)
    kt: int = field(init=False)
    kz: int = field(init=False)
    m: np.ndarray = field(init=False)       # m_j, j = 0..K_theta
    alpha: np.ndarray = field(init=False)   # alpha_l, l = -K_z..K_z
    w_outer: float = field(init=False)

    def __post_init__(self):
        g = self.geo
        g.validate()
        d = g.gap
        self.ri = d * g.zeta / (1.0 - g.zeta)
        self.ro = d / (1.0 - g.zeta)
        self.nu = d / g.re
        n = np.arange(g.nr, dtype=np.float64)
        xi = -1.0 + 2.0 * n / (g.nr - 1)
        if g.stretch > 0:
            # the C library's tanh point by point (numpy's vectorised tanh
            # can be one unit in the last place off, and the compact
            # coefficients of the clustered near-wall rows amplify a
            # one-ulp move of a grid point about a thousandfold)
            ts = math.tanh(g.stretch)
            t = np.array([math.tanh(g.stretch * x) for x in xi]) / ts
        else:
            t = xi
        self.r = self.ri + d * (1.0 + t) / 2.0
        self.r[0] = self.ri
        self.r[-1] = self.ro
        rc = 0.5 * (self.ri + self.ro)
        self.theta_period = g.theta_period if g.theta_period > 0 else min(2 * np.pi, 5 * np.pi * d / rc)
        self.lz = g.lz if g.lz > 0 else 2.5 * d
        self.kt = truncation(g.ntheta)
        self.kz = truncation(g.nz)
        self.m = 2 * np.pi * np.arange(self.kt + 1) / self.theta_period
        self.alpha = 2 * np.pi * np.arange(-self.kz, self.kz + 1) / self.lz
        # outer-wall azimuthal speed in units of W_i
        self.w_outer = g.re_outer / g.re

    @property
    def nj(self):
        return self.kt + 1

    @property
    def nl(self):
        return 2 * self.kz + 1

    def mode_arrays(self):
        """(m, alpha) broadcast to shape (1, nj, nl)."""
        m = self.m[None, :, None] * np.ones((1, 1, self.nl))
        al = self.alpha[None, None, :] * np.ones((1, self.nj, 1))
        return m, al
