"""Pins of the oracle's whole linear operator, time integrator and mean flow.

* Circular Couette flow (eq. (laminar-solution)) is the discrete steady state
  to fourth order in N_r (Sec. 3, Fig. 2), and its torque is Table 2's
  laminar value.
* The oracle's linearised operator about Couette flow (assembled column by
  column from the oracle's own functions) has its critical Reynolds number
  inside the paper's brackets (Sec. 3) and equal to an independent Chebyshev
  eigenproblem.
* An oracle DNS seeded with that eigenvector grows at the eigenvalue's rate
  (checks the RK3/CN integrator and the FFT products in the linear regime).
* The integrator converges at second order in dt.
"""

import os

import numpy as np
import pytest
from scipy.linalg import eig, solve_banded
from scipy.optimize import brentq

from oracle import Geometry, Oracle
from oracle import equations as eq
from oracle.stats import wall_shear
from tests.chebyshev_tc import growth_rate as cheb_growth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _steady_couette(orc):
    """Solve the oracle's discrete steady mean azimuthal equation L w = 0
    with w = 1 at the inner wall and W_o at the outer wall."""
    nr = orc.geo.nr
    R = orc.disc.r[:, None]
    ab = eq.band_terms(orc.ops, eq.wmean_visc_terms(R), 1)[0]
    for i, col in ((0, 0), (nr - 1, nr - 1)):
        for j in range(max(0, i - 3), min(nr, i + 4)):
            ab[3 + i - j, j] = 0.0
        ab[3, col] = 1.0
    rhs = np.zeros(nr)
    rhs[0], rhs[-1] = 1.0, orc.disc.w_outer
    return solve_banded((3, 3), ab, rhs)


def _laminar(r, zeta):
    ri = zeta / (1 - zeta)
    return (1.0 / (1 - zeta**2)) * (ri / r - zeta**2 * r / ri)


@pytest.mark.parametrize("stretch", [0.0, 1.5])
def test_couette_profile_converges_at_fourth_order(stretch):
    errs = []
    ns = (17, 33, 65)
    for n in ns:
        orc = Oracle(Geometry(zeta=0.5, re=60.0, nr=n, ntheta=4, nz=4, dt=1e-2, stretch=stretch))
        w = _steady_couette(orc)
        errs.append(np.max(np.abs(w - _laminar(orc.disc.r, 0.5))))
    p = np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert -5.5 < p < -3.5, (errs, p)
    assert errs[1] < 1e-5  # Fig. 2 range at N_r = 33


def test_laminar_torque_matches_table2():
    rows = np.loadtxt(os.path.join(GOLDEN, "table2_laminar_torque.txt"))
    for re, torque in rows:
        orc = Oracle(Geometry(zeta=0.5, re=re, nr=64, ntheta=4, nz=4, dt=1e-2))
        orc.w_mean = _steady_couette(orc)
        s = orc.stats()
        assert round(s["torque_in"], 4) == torque
        assert abs(s["torque_out"] / s["torque_in"] - 1) < 1e-5
        # laminar shear scales as 1/r^2, so Re_tau,o / Re_tau,i = zeta (Sec. 5)
        assert abs(s["retau_out"] / s["retau_in"] - 0.5) < 1e-5


def test_steady_couette_is_a_fixed_point_of_the_step():
    orc = Oracle(Geometry(zeta=0.883, re=150.0, nr=33, ntheta=8, nz=8, dt=1e-2))
    w = _steady_couette(orc)
    orc.load(np.zeros((33, orc.disc.nj, orc.disc.nl)), np.zeros((33, orc.disc.nj, orc.disc.nl)),
             np.zeros(33), w)
    orc.step(3)
    v, e, um, wm = orc.fields()
    assert np.max(np.abs(wm - w)) < 1e-13
    assert np.max(np.abs(um)) == 0.0
    assert np.max(np.abs(v)) == 0.0 and np.max(np.abs(e)) == 0.0


def linear_operator(orc, j, l, wbase):
    """Matrices (A, B) of the semi-discrete linearised system B dq/dt = A q
    for the mode (j, l), q = (v, eta) on all N_r points, with the boundary
    rows of the oracle's solves (A row = constraint, B row = 0).  Built by
    applying the oracle's own operators to unit vectors; the products are
    linearised about the mean flow w_base: uw = W u, vw = W v, ww = 2 W w."""
    nr = orc.geo.nr
    kz = orc.disc.kz
    m = np.array([orc.disc.m[j]])
    al = np.array([orc.disc.alpha[l + kz]])
    mc = eq.ModeCoefficients(orc.disc.r, m, al)
    ops = orc.ops
    nu = orc.disc.nu
    W = wbase[:, None]
    A = np.zeros((2 * nr, 2 * nr), dtype=complex)
    B = np.zeros((2 * nr, 2 * nr), dtype=complex)
    for i in range(2 * nr):
        v = np.zeros((nr, 1), dtype=complex)
        e = np.zeros((nr, 1), dtype=complex)
        (v if i < nr else e)[i % nr] = 1.0
        dv = ops.radial_derivative(v)
        u, w, c = eq.recover_velocity(ops, mc, v, e, dv)
        z = np.zeros_like(v)
        P = {"uu": z, "uv": z, "uw": W * u, "vv": z, "vw": W * v, "ww": 2 * W * w}
        nv = nu * eq.v_explicit_viscous(ops, mc, u, w, c) + eq.v_nonlinear(ops, mc, P)
        ne = nu * eq.eta_explicit_viscous(ops, mc, u, v) + eq.eta_nonlinear(ops, mc, P)
        A[:nr, i] = (nu * eq.apply_terms(ops, eq.v_visc_terms(mc), v) + nv)[:, 0]
        A[nr:, i] = (nu * eq.apply_terms(ops, eq.eta_visc_terms(mc), e) + ne)[:, 0]
        B[:nr, i] = eq.apply_terms(ops, eq.v_mass_terms(mc), v)[:, 0]
        B[nr:, i] = eq.apply_terms(ops, eq.eta_mass_terms(mc), e)[:, 0]
    d1 = orc.coef["d1"]
    cons = {0: {0: 1.0}, 1: dict(enumerate(d1[0])),
            nr - 2: {nr - 5 + k: d1[nr - 1][k] for k in range(5)}, nr - 1: {nr - 1: 1.0},
            nr: {nr: 1.0}, 2 * nr - 1: {2 * nr - 1: 1.0}}
    for row, entries in cons.items():
        A[row] = 0
        B[row] = 0
        for col, val in entries.items():
            A[row, col] = val
    return A, B


def _oracle_growth(zeta, re, nr=33):
    orc = Oracle(Geometry(zeta=zeta, re=re, nr=nr, ntheta=4, nz=4, dt=1e-2, lz=2.0))
    wbase = _steady_couette(orc)
    A, B = linear_operator(orc, 0, 1, wbase)
    lam, vec = eig(A, B)
    ok = np.isfinite(lam) & (np.abs(lam) < 1e6)
    k = np.argmax(np.where(ok, lam.real, -np.inf))
    return lam[k], vec[:, k], orc, wbase


def test_critical_reynolds_numbers_match_paper_and_chebyshev():
    rows = np.loadtxt(os.path.join(GOLDEN, "critical_reynolds.txt"))
    for zeta, lo, hi in rows:
        rec = brentq(lambda re: _oracle_growth(zeta, re)[0].real, lo - 10, hi + 10, xtol=1e-6)
        ref = brentq(lambda re: cheb_growth(zeta, re, np.pi, 40), lo - 10, hi + 10, xtol=1e-6)
        assert lo < rec < hi, (zeta, rec)
        assert abs(rec / ref - 1) < 1e-3, (zeta, rec, ref)


def test_growth_rate_matches_chebyshev_away_from_onset():
    for re in (50.0, 90.0):
        lam = _oracle_growth(0.5, re)[0]
        ref = cheb_growth(0.5, re, np.pi, 40)
        assert abs(lam.real - ref) < 2e-4, (re, lam, ref)


def _seed_eigenvector(orc, vec, amp):
    nr = orc.geo.nr
    kz = orc.disc.kz
    v = np.zeros((nr, orc.disc.nj, orc.disc.nl), dtype=complex)
    e = np.zeros_like(v)
    scale = amp / np.max(np.abs(vec[:nr]))
    v[:, 0, kz + 1] = vec[:nr] * scale
    e[:, 0, kz + 1] = vec[nr:] * scale
    v[:, 0, kz - 1] = np.conj(v[:, 0, kz + 1])
    e[:, 0, kz - 1] = np.conj(e[:, 0, kz + 1])
    v[[0, -1]] = 0
    e[[0, -1]] = 0
    return v, e


def test_dns_grows_at_the_eigenvalue_rate():
    lam, vec, orc, wbase = _oracle_growth(0.5, 80.0)
    assert lam.real > 0 and abs(lam.imag) < 1e-8  # exchange of stabilities
    v, e = _seed_eigenvector(orc, vec, 1e-6)
    orc.load(v, e, np.zeros(orc.geo.nr), wbase)
    e0 = orc.stats()["energy_pert"]
    orc.step(100)  # t = 1
    e1 = orc.stats()["energy_pert"]
    sigma = np.log(e1 / e0) / (2 * 1.0)
    assert abs(sigma / lam.real - 1) < 1e-4, (sigma, lam)


def test_time_integration_is_second_order():
    geo = dict(zeta=0.5, re=60.0, nr=25, ntheta=4, nz=4, lz=2.0)
    lam, vec, orc, wbase = _oracle_growth(0.5, 60.0, nr=25)
    # start from a non-eigen state: the leading mode plus a second mode
    v, e = _seed_eigenvector(orc, vec, 1e-6)
    v2 = v.copy()
    rng = np.random.default_rng(0)
    x = (2 * orc.disc.r - orc.disc.ri - orc.disc.ro)
    v2[:, 0, 2] += 1e-6 * (1 - x**2) ** 2 * (1 + 0.5j)
    v2[:, 0, 0] = np.conj(v2[:, 0, 2])
    finals = []
    for dt in (0.2, 0.1, 0.05, 0.0125):
        o = Oracle(Geometry(dt=dt, **geo))
        o.load(v2, e, np.zeros(25), wbase)
        o.step(int(round(2.0 / dt)))
        finals.append(o.fields()[0])
    ref = finals[-1]
    err = [np.max(np.abs(f - ref)) for f in finals[:-1]]
    ratios = [err[0] / err[1], err[1] / err[2]]
    assert all(3.3 < q < 4.8 for q in ratios), (err, ratios)
