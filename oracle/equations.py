"""Velocity recovery, right-hand sides and mean-mode equations (oracle side).

Fields are handled "mode-flattened": shape (N_r, M) for M Fourier modes whose
azimuthal and axial wavenumbers are given by arrays m, alpha of shape (M,).

Notation (Appendix): D f = df/dr, D_* f = df/dr + f/r, k^2 = alpha^2 + m^2/r^2,
a = 1/k^2 with a1, a2, a3 its first three analytic r-derivatives (the "known
coefficients" that integration by parts introduces, such as D(1/k^2)).
[g]_L denotes the compact operator family L applied to g (see ``compact``);
a bare term g is [g]_0.

Implicit/explicit split (reading of Sec. 2.1 and the Appendix): viscous terms
acting on v alone (eta alone) are implicit (Crank--Nicolson); the
curvature-related viscous terms that involve u or w, including those created
by the continuity substitution, are explicit together with the nonlinear
terms.
"""

import numpy as np
from scipy.linalg import solve_banded

from .compact import apply as compact_apply


class ModeCoefficients:
    """a = 1/k^2 and its analytic derivatives on the grid, for M modes.

    With s = alpha^2 r^2 + m^2 (so a = r^2/s):
        a1 = 2 m^2 r / s^2
        a2 = 2 m^2 (m^2 - 3 alpha^2 r^2) / s^3
        a3 = -24 m^2 alpha^2 r (m^2 - alpha^2 r^2) / s^4
    The (0,0) mode has no such coefficients; its entries are set to harmless
    dummies and the mean flow is treated separately.
    """

    def __init__(self, r, m, alpha):
        R = np.asarray(r, dtype=np.float64)[:, None]
        m = np.asarray(m, dtype=np.float64)[None, :]
        al = np.asarray(alpha, dtype=np.float64)[None, :]
        self.is_mean = ((m == 0) & (al == 0))[0]
        s = al**2 * R**2 + m**2
        s = np.where(self.is_mean[None, :], 1.0, s)
        self.R = R
        self.m = m
        self.alpha = al
        self.k2 = s / R**2
        self.a = R**2 / s
        self.a1 = 2 * m**2 * R / s**2
        self.a2 = 2 * m**2 * (m**2 - 3 * al**2 * R**2) / s**3
        self.a3 = -24 * m**2 * al**2 * R * (m**2 - al**2 * R**2) / s**4


class Operators:
    """Compact operators of one grid: [g]_L for L in d0, d1, d2, d2s, d4s."""

    def __init__(self, coef, sigma):
        self.coef = coef
        self.sigma = sigma
        self.nr = sigma.size

    def __call__(self, fam, g):
        return compact_apply(self.coef[fam], self.sigma, g)

    # --- recovery (Appendix: continuity substitution) -------------------
    def radial_derivative(self, v):
        """Dv from sum_j d0[n,j] Dv_{sigma+j} = sum_j d1[n,j] v_{sigma+j} on
        rows 1..N_r-2, with Dv = 0 at both walls (no-slip, Appendix).  The
        d0 block on rows 1..N_r-2 is pentadiagonal; solved with LAPACK."""
        nr = self.nr
        rhs = self("d1", v)[1:nr - 1]
        ab = np.zeros((5, nr - 2))
        d0 = self.coef["d0"]
        for n in range(1, nr - 1):
            for j in range(5):
                col = self.sigma[n] + j
                if 1 <= col <= nr - 2 and d0[n, j] != 0.0:
                    ab[2 + (n - 1) - (col - 1), col - 1] = d0[n, j]
        dv = np.zeros_like(v)
        dv[1:nr - 1] = solve_banded((2, 2), ab, rhs)
        return dv


def recover_velocity(ops, mc, v, eta, dv):
    """u and w from v, eta through continuity D_* v = -i alpha u - (i m / r) w
    and the definition eta = (i m / r) u - i alpha w (Appendix):

        u = (i alpha D_* v - (i m / r) eta) / k^2
        w = ((i m / r) D_* v + i alpha eta) / k^2

    Returns (u, w, c) with c = i alpha u + (i m / r) w (= -D_* v)."""
    dsv = dv + v / mc.R
    im_r = 1j * mc.m / mc.R
    ia = 1j * mc.alpha
    u = (ia * dsv - im_r * eta) * mc.a
    w = (im_r * dsv + ia * eta) * mc.a
    u[:, mc.is_mean] = 0.0
    w[:, mc.is_mean] = 0.0
    c = ia * u + im_r * w
    return u, w, c


# --- implicit operators, written as (family, coefficient) term lists -------
# A term (L, g) stands for [g q]_L applied to the unknown q.

def v_mass_terms(mc):
    """Time-derivative operator of eq. (final-v):
    v - D D_*(v/k^2) + D(v D(1/k^2))."""
    return [("d0", 1.0), ("d2s", -mc.a), ("d1", mc.a1)]


def v_visc_terms(mc):
    """Viscous terms of eq. (final-v) that act on v alone (implicit):
    2 D D_* v - D D_* D D_*(v/k^2) + D[(1/r) DD(1/k^2) v]
    - 2 D D_*[(1/r) D(1/k^2) v] + D[DDD(1/k^2) v] - D[(1/r^2) D(1/k^2) v]
    - 2 m^2 D(v/(k^2 r^3)) - k^2 v."""
    R = mc.R
    return [("d2s", 2.0), ("d4s", -mc.a), ("d1", mc.a2 / R), ("d2s", -2 * mc.a1 / R),
            ("d1", mc.a3), ("d1", -mc.a1 / R**2), ("d1", -2 * mc.m**2 * mc.a / R**3),
            ("d0", -mc.k2)]


def eta_mass_terms(mc):
    return [("d0", 1.0)]


def eta_visc_terms(mc):
    """Viscous terms of eq. (final-eta) acting on eta alone: D D_* eta - k^2 eta."""
    return [("d2s", 1.0), ("d0", -mc.k2)]


def umean_visc_terms(R):
    """Mean axial velocity (k = 0 limit of the axial momentum equation):
    D_* D u = D D_* u + u / r^2."""
    return [("d2s", 1.0), ("d0", 1.0 / R**2)]


def wmean_visc_terms(R):
    """Mean azimuthal velocity: D_* D w - w / r^2 = D D_* w."""
    return [("d2s", 1.0)]


def mass_terms_identity():
    return [("d0", 1.0)]


def apply_terms(ops, terms, q):
    out = np.zeros(q.shape, dtype=np.result_type(q, np.float64))
    for fam, g in terms:
        out += ops(fam, g * q)
    return out


def band_terms(ops, terms, nmodes, kl=3, ku=3):
    """Banded (LAPACK layout) matrix of a sum of terms, one per mode:
    ab[mode, ku + i - j, j] = A[i, j] with A[n, sigma_n + j] += dL[n, j] g(r_{sigma_n + j}).
    Only the rows 1..N_r-2 are assembled (the wall rows are boundary
    conditions); their entries lie within three diagonals of the main one."""
    nr = ops.nr
    ab = np.zeros((nmodes, kl + ku + 1, nr))
    rows = np.arange(1, nr - 1)
    for fam, g in terms:
        c = ops.coef[fam]
        garr = np.broadcast_to(np.asarray(g, dtype=np.float64), (nr, nmodes))
        for j in range(5):
            cols = ops.sigma[rows] + j
            ab[:, ku + rows - cols, cols] += (c[rows, j][:, None] * garr[cols]).T
    return ab


# --- explicit terms -------------------------------------------------------

def v_explicit_viscous(ops, mc, u, w, c):
    """Explicit viscous terms of eq. (final-v) (curvature terms through u, w
    and the term created by the continuity substitution):
    -3 D D_*[D(1/k^2) c] + 2im D[w/(k^2 r^3)]
    + 2im (DD[w/(k^2 r^2)] - D[(1/r^2) D(1/k^2) w]) - 2 (im/r^2) w."""
    R = mc.R
    im = 1j * mc.m
    return (-3 * ops("d2s", mc.a1 * c)
            + 2 * im * ops("d1", mc.a * w / R**3)
            + 2 * im * (ops("d2", mc.a * w / R**2) - ops("d1", mc.a1 * w / R**2))
            - 2 * im * ops("d0", w / R**2))


def v_nonlinear(ops, mc, P):
    """Nonlinear terms of eq. (final-v), from the product spectra P."""
    R = mc.R
    ia = 1j * mc.alpha
    im = 1j * mc.m
    al = mc.alpha
    m = mc.m
    a, a1 = mc.a, mc.a1
    UU, UV, UW, VV, VW, WW = (P[k] for k in ("uu", "uv", "uw", "vv", "vw", "ww"))
    return (-ia * (ops("d2s", a * UV) - ops("d1", a1 * UV))
            - im * (ops("d2", a * VW / R) + 3 * ops("d1", a * VW / R**2) - ops("d1", a1 * VW / R))
            + ops("d1", a * (al**2 * UU + 2 * (al * m / R) * UW + (m**2 / R**2) * WW))
            - ia * ops("d0", UV) - ops("d1", VV) - im * ops("d0", VW / R)
            - ops("d0", VV / R) + ops("d0", WW / R))


def eta_explicit_viscous(ops, mc, u, v):
    """Explicit viscous terms of eq. (final-eta):
    2im [D(u/r^2) + 2 u/r^3 - (i alpha / r^2) v]."""
    R = mc.R
    im = 1j * mc.m
    ia = 1j * mc.alpha
    return 2 * im * (ops("d1", u / R**2) + 2 * ops("d0", u / R**3) - ia * ops("d0", v / R**2))


def eta_nonlinear(ops, mc, P):
    """Nonlinear terms of eq. (final-eta)."""
    R = mc.R
    im = 1j * mc.m
    ia = 1j * mc.alpha
    UU, UV, UW, VV, VW, WW = (P[k] for k in ("uu", "uv", "uw", "vv", "vw", "ww"))
    return (-im * (ia * ops("d0", UU / R) + ops("d1", UV / R) + 2 * ops("d0", UV / R**2)
                   + im * ops("d0", UW / R**2))
            + ia * (ia * ops("d0", UW) + ops("d1", VW) + im * ops("d0", WW / R)
                    + 2 * ops("d0", VW / R)))


def umean_nonlinear(ops, R, uv00):
    """Mean axial momentum with null mean pressure gradient (Sec. 4):
    -D_*(UV) at k = 0, i.e. -(D(UV) + UV/r)."""
    return -(ops("d1", uv00) + ops("d0", uv00 / R))


def wmean_nonlinear(ops, R, vw00):
    """Mean azimuthal momentum: -(D(VW) + 2 VW / r)."""
    return -(ops("d1", vw00) + 2 * ops("d0", vw00 / R))
