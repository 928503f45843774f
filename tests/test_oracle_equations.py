"""Pins of the oracle's discrete equations against the mathematics.

Each discrete operator of the oracle (a d0-multiplied row, see the compact
scheme) is applied to smooth manufactured fields on one Fourier mode and
compared with d0 applied to the exact operator evaluated in closed form from
the primitive-variable cylindrical Navier--Stokes equations (tests/analytic.py).
A dropped term, a wrong sign or a wrong index in eq. (final-v),
eq. (final-eta), the recovery or the mean-flow equations leaves an O(1)
error; the correct discretisation converges at the scheme's order.
"""

import numpy as np
import pytest
import sympy as sp

from oracle import equations as eq
from oracle.compact import compact_coefficients
from tests.analytic import Mode, MeanProfiles


def _grid(n, ri=1.0, ro=2.0, stretch=1.2):
    xi = -1 + 2 * np.arange(n) / (n - 1)
    t = np.tanh(stretch * xi) / np.tanh(stretch)
    r = ri + (ro - ri) * (1 + t) / 2
    r[0], r[-1] = ri, ro
    return r


def _errors(n, mode):
    r = _grid(n)
    coef, sigma = compact_coefficients(r)
    ops = eq.Operators(coef, sigma)
    mc = eq.ModeCoefficients(r, np.array([mode.m]), np.array([mode.alpha]))
    col = lambda x: x[:, None]
    F = {k: col(f(r)) for k, f in mode.f.items()}
    d0 = lambda t: ops("d0", col(mode.t[t](r)))
    out = {}
    v_mass = eq.apply_terms(ops, eq.v_mass_terms(mc), F["v"])
    v_visc = (eq.apply_terms(ops, eq.v_visc_terms(mc), F["v"])
              + eq.v_explicit_viscous(ops, mc, F["u"], F["w"], F["c"]))
    v_nl = eq.v_nonlinear(ops, mc, F)
    e_visc = (eq.apply_terms(ops, eq.eta_visc_terms(mc), F["eta"])
              + eq.eta_explicit_viscous(ops, mc, F["u"], F["v"]))
    e_nl = eq.eta_nonlinear(ops, mc, F)
    vr = slice(2, n - 2)
    er = slice(1, n - 1)
    for name, disc, rows in (("v_mass", v_mass, vr), ("v_visc", v_visc, vr), ("v_nl", v_nl, vr),
                             ("eta_visc", e_visc, er), ("eta_nl", e_nl, er)):
        ref = d0(name)
        out[name] = np.max(np.abs(disc[rows] - ref[rows])) / np.max(np.abs(ref[rows]))
    # recovery: u and w from (v, eta) through the compact derivative
    dv = ops.radial_derivative(F["v"])
    u, w, c = eq.recover_velocity(ops, mc, F["v"], F["eta"], dv)
    out["u"] = np.max(np.abs(u - F["u"])) / np.max(np.abs(F["u"]))
    out["w"] = np.max(np.abs(w - F["w"])) / np.max(np.abs(F["w"]))
    return out


@pytest.mark.parametrize("alpha,m", [(1.3, 2.7), (2.0, 0.0), (0.0, 3.0)])
def test_final_equations_converge_to_primitive_navier_stokes(alpha, m):
    mode = Mode(1.0, 2.0, alpha, m)
    e1 = _errors(33, mode)
    e2 = _errors(65, mode)
    for k in e1:
        order = np.log2(e1[k] / e2[k]) if e2[k] > 0 else 99
        # every operator is at least third order on this stretched grid and
        # already small on the finer grid
        assert e2[k] < 2e-4, (k, e2[k])
        if e1[k] > 1e-12:  # polynomial fields are reproduced exactly
            assert order > 2.7, (k, e1[k], e2[k], order)


def test_mean_flow_operators():
    r_i, r_o = 1.0, 2.0
    prof = MeanProfiles(r_i, r_o)
    errs = []
    for n in (33, 65):
        r = _grid(n)
        R = r[:, None]
        coef, sigma = compact_coefficients(r)
        ops = eq.Operators(coef, sigma)
        col = lambda x: np.real(x)[:, None]
        um, wm = col(prof.f["u"](r)), col(prof.f["w"](r))
        uv, vw = col(prof.f["uv"](r)), col(prof.f["vw"](r))
        got = {
            "u_visc": eq.apply_terms(ops, eq.umean_visc_terms(R), um),
            "w_visc": eq.apply_terms(ops, eq.wmean_visc_terms(R), wm),
            "u_nl": eq.umean_nonlinear(ops, R, uv),
            "w_nl": eq.wmean_nonlinear(ops, R, vw),
        }
        rows = slice(1, n - 1)
        e = {}
        for k, g in got.items():
            ref = ops("d0", col(prof.t[k](r)))
            e[k] = np.max(np.abs(g[rows] - ref[rows])) / np.max(np.abs(ref[rows]))
        errs.append(e)
    for k in errs[0]:
        assert errs[1][k] < 1e-4, (k, errs[1][k])
        assert np.log2(errs[0][k] / errs[1][k]) > 2.7, k


def test_wavenumber_coefficients_are_derivatives_of_inverse_k2():
    """a1, a2, a3 are the analytic r-derivatives of 1/k^2 (checked with sympy)."""
    rs = sp.Symbol("r", positive=True)
    r = np.linspace(1.0, 2.0, 7)
    for al, m in ((1.3, 2.7), (0.0, 2.0), (3.0, 0.0), (0.4, 5.0)):
        a = 1 / (sp.nsimplify(al) ** 2 + sp.nsimplify(m) ** 2 / rs**2)
        mc = eq.ModeCoefficients(r, np.array([m]), np.array([al]))
        for k, got in enumerate((mc.a, mc.a1, mc.a2, mc.a3)):
            ref = np.array([float(sp.diff(a, rs, k).subs(rs, x)) for x in r])
            np.testing.assert_allclose(got[:, 0], ref, rtol=1e-12, atol=1e-14)


def test_band_assembly_matches_operator_application():
    """The banded matrices the implicit solves use are the same linear maps as
    the term lists applied directly (rows 1..N_r-2)."""
    r = _grid(21)
    coef, sigma = compact_coefficients(r)
    ops = eq.Operators(coef, sigma)
    mc = eq.ModeCoefficients(r, np.array([1.7, 0.0]), np.array([0.9, 2.2]))
    rng = np.random.default_rng(5)
    q = rng.standard_normal((21, 2))
    for terms in (eq.v_mass_terms(mc), eq.v_visc_terms(mc), eq.eta_visc_terms(mc)):
        ab = eq.band_terms(ops, terms, 2)
        direct = eq.apply_terms(ops, terms, q)
        for i in range(2):
            dense = np.zeros((21, 21))
            for row in range(21):
                for col in range(max(0, row - 3), min(21, row + 4)):
                    dense[row, col] = ab[i, 3 + row - col, col]
            np.testing.assert_allclose((dense @ q[:, i])[1:-1], direct[1:-1, i], rtol=1e-12, atol=1e-9)
