"""One RK3 / Crank--Nicolson substep of the Taylor--Couette DNS (oracle side).

Sec. 2.1 and Sec. 3.1: a 3-substep Runge--Kutta scheme, explicit for the
nonlinear and curvature-related viscous terms, with a second-order
Crank--Nicolson scheme for the remaining viscous terms.  The coefficients are
not printed; the reading taken is the low-storage scheme

    (M - b_k dt nu L) q^k = (M + b_k dt nu L) q^{k-1}
                            + dt (g_k N^{k-1} + p_k N^{k-2}),

with g = (8/15, 5/12, 3/4), p = (0, -17/60, -5/12) and equal implicit and
explicit Crank--Nicolson weights b_k = (g_k + p_k)/2 = (4/15, 1/15, 1/6), for
q in {v, eta, mean u, mean w}.  N = nu E + NL collects the explicit viscous
and nonlinear terms; every row of M, L and N is the d0-multiplied discrete
equation (see ``compact``).

Boundary conditions (Appendix): v = D v = eta = 0 at both walls.  The v system
uses rows 0 and N_r-1 for v = 0, rows 1 and N_r-2 for the wall derivative
conditions sum_j d1[0, j] v_j = 0 and sum_j d1[N_r-1, j] v_{N_r-5+j} = 0, and
its equation rows 2..N_r-3; eta has Dirichlet rows 0, N_r-1 and equation rows
1..N_r-2.  Mean flow (Sec. 4: null mean pressure gradient in both homogeneous
directions): u = 0 at both walls, w = 1 on the inner and W_o on the outer
wall, equation rows 1..N_r-2.  All systems are solved with LAPACK's banded LU
with partial pivoting (kl = ku = 3).
"""

import numpy as np
from scipy.linalg import solve_banded

from . import equations as eq
from .compact import compact_coefficients
from .grid import Discretisation
from .spectral import products as spectral_products
from . import stats as st

GAMMA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
RHO = (0.0, -17.0 / 60.0, -5.0 / 12.0)
BETA = tuple(0.5 * (g + r) for g, r in zip(GAMMA, RHO))

KL = KU = 3


def _set_row(ab, i, cols, vals):
    """Replace row i of banded matrices ab (modes, 7, nr) by vals at cols."""
    nr = ab.shape[2]
    for j in range(max(0, i - KL), min(nr, i + KU + 1)):
        ab[:, KU + i - j, j] = 0.0
    for c, v in zip(cols, vals):
        ab[:, KU + i - c, c] = v


def _solve_each(ab, rhs):
    """Solve ab[i] x = rhs[:, i] for every mode i (complex rhs, real matrix)."""
    nr, nm = rhs.shape
    out = np.empty_like(rhs)
    for i in range(nm):
        b = np.stack([rhs[:, i].real, rhs[:, i].imag], axis=1)
        x = solve_banded((KL, KU), ab[i], b, check_finite=False)
        out[:, i] = x[:, 0] + 1j * x[:, 1]
    return out


class Oracle:
    """FP64 CPU reference solver of one Taylor--Couette instance."""

    def __init__(self, geo):
        self.geo = geo
        self.disc = Discretisation(geo)
        d = self.disc
        self.coef, self.sigma = compact_coefficients(d.r)
        self.ops = eq.Operators(self.coef, self.sigma)
        m, al = d.mode_arrays()
        self.m_flat = m.reshape(-1)
        self.alpha_flat = al.reshape(-1)
        self.mc = eq.ModeCoefficients(d.r, self.m_flat, self.alpha_flat)
        self.mean_index = int(np.flatnonzero(self.mc.is_mean)[0])
        self.nmodes = d.nj * d.nl
        nr = geo.nr
        self.v = np.zeros((nr, self.nmodes), dtype=np.complex128)
        self.eta = np.zeros_like(self.v)
        self.u_mean = np.zeros(nr)
        self.w_mean = np.zeros(nr)
        self.time = 0.0
        self.steps = 0
        self._zero_registers()

    # ------------------------------------------------------------------ I/O
    def _zero_registers(self):
        self.nv_prev = np.zeros_like(self.v)
        self.neta_prev = np.zeros_like(self.v)
        self.nu_prev = np.zeros(self.geo.nr)
        self.nw_prev = np.zeros(self.geo.nr)

    def load(self, v, eta, u_mean, w_mean):
        """Load spectral fields [r][j][l + K_z] and the mean profiles."""
        d = self.disc
        shape = (self.geo.nr, d.nj, d.nl)
        v = np.asarray(v, dtype=np.complex128).reshape(shape)
        eta = np.asarray(eta, dtype=np.complex128).reshape(shape)
        self.v = v.reshape(self.geo.nr, -1).copy()
        self.eta = eta.reshape(self.geo.nr, -1).copy()
        self.u_mean = np.asarray(u_mean, dtype=np.float64).copy()
        self.w_mean = np.asarray(w_mean, dtype=np.float64).copy()
        self._zero_registers()

    def fields(self):
        d = self.disc
        shape = (self.geo.nr, d.nj, d.nl)
        return (self.v.reshape(shape).copy(), self.eta.reshape(shape).copy(),
                self.u_mean.copy(), self.w_mean.copy())

    # ------------------------------------------------------------ pieces
    def velocity(self, v=None, eta=None, u_mean=None, w_mean=None):
        """(dv, u, w, c) for all modes, with the mean flow in the (0,0) slot
        of u and w."""
        v = self.v if v is None else v
        eta = self.eta if eta is None else eta
        u_mean = self.u_mean if u_mean is None else u_mean
        w_mean = self.w_mean if w_mean is None else w_mean
        dv = self.ops.radial_derivative(v)
        u, w, c = eq.recover_velocity(self.ops, self.mc, v, eta, dv)
        u[:, self.mean_index] = u_mean
        w[:, self.mean_index] = w_mean
        return dv, u, w, c

    def products(self, u, v, w):
        d = self.disc
        shape = (self.geo.nr, d.nj, d.nl)
        P = spectral_products(u.reshape(shape), v.reshape(shape), w.reshape(shape),
                              self.geo.ntheta, self.geo.nz)
        return {k: x.reshape(self.geo.nr, -1) for k, x in P.items()}

    def _sub_mc(self, idx):
        return eq.ModeCoefficients(self.disc.r, self.m_flat[idx], self.alpha_flat[idx])

    def explicit_terms(self, idx, u, v, w, c, P):
        """N = nu E + NL for v and eta on the modes idx (rows all r)."""
        mc = self._sub_mc(idx)
        ops = self.ops
        nu = self.disc.nu
        Ps = {k: x[:, idx] for k, x in P.items()}
        nv = nu * eq.v_explicit_viscous(ops, mc, u[:, idx], w[:, idx], c[:, idx]) + eq.v_nonlinear(ops, mc, Ps)
        ne = nu * eq.eta_explicit_viscous(ops, mc, u[:, idx], v[:, idx]) + eq.eta_nonlinear(ops, mc, Ps)
        return nv, ne

    def lhs_v(self, mc, bdt_nu):
        nr = self.geo.nr
        terms = eq.v_mass_terms(mc) + [(f, -bdt_nu * g) for f, g in eq.v_visc_terms(mc)]
        ab = eq.band_terms(self.ops, terms, mc.a.shape[1], KL, KU)
        d1 = self.coef["d1"]
        _set_row(ab, 0, [0], [1.0])
        _set_row(ab, 1, range(0, 5), d1[0])
        _set_row(ab, nr - 2, range(nr - 5, nr), d1[nr - 1])
        _set_row(ab, nr - 1, [nr - 1], [1.0])
        return ab

    def lhs_eta(self, mc, bdt_nu):
        nr = self.geo.nr
        terms = eq.eta_mass_terms(mc) + [(f, -bdt_nu * g) for f, g in eq.eta_visc_terms(mc)]
        ab = eq.band_terms(self.ops, terms, mc.a.shape[1], KL, KU)
        _set_row(ab, 0, [0], [1.0])
        _set_row(ab, nr - 1, [nr - 1], [1.0])
        return ab

    def lhs_mean(self, visc_terms, bdt_nu):
        nr = self.geo.nr
        terms = eq.mass_terms_identity() + [(f, -bdt_nu * g) for f, g in visc_terms]
        ab = eq.band_terms(self.ops, terms, 1, KL, KU)
        _set_row(ab, 0, [0], [1.0])
        _set_row(ab, nr - 1, [nr - 1], [1.0])
        return ab

    def radial_update(self, k, idx, v, eta, nv, ne, nv_prev, ne_prev):
        """Solve the substep-k systems for v and eta on the modes idx."""
        nr = self.geo.nr
        dt = self.geo.dt
        bdt_nu = BETA[k] * dt * self.disc.nu
        mc = self._sub_mc(idx)
        ops = self.ops
        vq = v[:, idx]
        eq_ = eta[:, idx]
        rv = (eq.apply_terms(ops, eq.v_mass_terms(mc), vq)
              + bdt_nu * eq.apply_terms(ops, eq.v_visc_terms(mc), vq)
              + dt * (GAMMA[k] * nv + RHO[k] * nv_prev))
        re_ = (eq.apply_terms(ops, eq.eta_mass_terms(mc), eq_)
               + bdt_nu * eq.apply_terms(ops, eq.eta_visc_terms(mc), eq_)
               + dt * (GAMMA[k] * ne + RHO[k] * ne_prev))
        rv[[0, 1, nr - 2, nr - 1]] = 0.0
        re_[[0, nr - 1]] = 0.0
        new_v = _solve_each(self.lhs_v(mc, bdt_nu), rv)
        new_e = _solve_each(self.lhs_eta(mc, bdt_nu), re_)
        return new_v, new_e

    def mean_update(self, k, P, u_mean, w_mean, nu_prev, nw_prev):
        """Mean (0,0) mode: mean axial and azimuthal velocity profiles, forced
        by the (0,0) coefficients of uv and vw (Sec. 4)."""
        nr = self.geo.nr
        dt = self.geo.dt
        bdt_nu = BETA[k] * dt * self.disc.nu
        R = self.disc.r[:, None]
        ops = self.ops
        uv00 = P["uv"][:, self.mean_index].real[:, None]
        vw00 = P["vw"][:, self.mean_index].real[:, None]
        n_u = eq.umean_nonlinear(ops, R, uv00)[:, 0]
        n_w = eq.wmean_nonlinear(ops, R, vw00)[:, 0]
        out = []
        for q, visc, nq, nprev, walls in (
                (u_mean, eq.umean_visc_terms(R), n_u, nu_prev, (0.0, 0.0)),
                (w_mean, eq.wmean_visc_terms(R), n_w, nw_prev, (1.0, self.disc.w_outer))):
            qc = q[:, None]
            rhs = (ops("d0", qc)[:, 0] + bdt_nu * eq.apply_terms(ops, visc, qc)[:, 0]
                   + dt * (GAMMA[k] * nq + RHO[k] * nprev))
            rhs[0], rhs[nr - 1] = walls
            ab = self.lhs_mean(visc, bdt_nu)[0]
            out.append(solve_banded((KL, KU), ab, rhs, check_finite=False))
        return out[0], out[1], n_u, n_w

    # ------------------------------------------------------------- stepping
    def substep(self, k):
        """Advance the state by substep k in {0, 1, 2} (the paper's 1, 2, 3)."""
        dv, u, w, c = self.velocity()
        P = self.products(u, self.v, w)
        idx = np.flatnonzero(~self.mc.is_mean)
        nv, ne = self.explicit_terms(idx, u, self.v, w, c, P)
        new_v, new_e = self.radial_update(k, idx, self.v, self.eta, nv, ne,
                                          self.nv_prev[:, idx], self.neta_prev[:, idx])
        um, wm, n_u, n_w = self.mean_update(k, P, self.u_mean, self.w_mean,
                                            self.nu_prev, self.nw_prev)
        self.v[:, idx] = new_v
        self.eta[:, idx] = new_e
        self.nv_prev[:, idx] = nv
        self.neta_prev[:, idx] = ne
        self.u_mean, self.w_mean = um, wm
        self.nu_prev, self.nw_prev = n_u, n_w

    def step(self, nsteps=1):
        for _ in range(nsteps):
            for k in range(3):
                self.substep(k)
            self.time += self.geo.dt
            self.steps += 1

    def substep_sample(self, k, modes):
        """Substep k from the current state for the listed flat mode indices
        only, without changing the state: returns (v_new, eta_new) of shape
        (N_r, len(modes)).  Used to check large grids on a sample of modes;
        the products are still evaluated on the whole grid."""
        modes = np.asarray(modes)
        if np.any(self.mc.is_mean[modes]):
            raise ValueError("the (0,0) mode is the mean flow")
        dv, u, w, c = self.velocity()
        P = self.products(u, self.v, w)
        nv, ne = self.explicit_terms(modes, u, self.v, w, c, P)
        return self.radial_update(k, modes, self.v, self.eta, nv, ne,
                                  self.nv_prev[:, modes], self.neta_prev[:, modes])

    # ---------------------------------------------------------------- stats
    def stats(self):
        dv, u, w, c = self.velocity()
        return st.statistics(self, u, w)

    def profiles(self):
        dv, u, w, c = self.velocity()
        return st.plane_profiles(self, u, w)
