"""Pins of the oracle's compact finite-difference coefficients.

* Planar uniform limit: far from the axis on a uniform grid the construction
  must give the classical compact fourth-derivative scheme (denominator
  (-1, 124, 474, 124, -1)/720 with numerator (1, -4, 6, -4, 1)/h^4) and the
  matching second- and first-derivative rows (1, 8, -18, 8, 1)/(12 h^2) and
  (0, -1/2, 0, 1/2, 0)/h.
* Local truncation order on non-polynomial functions on a stretched grid.
* Near-wall rows are explicit (d0 = e_n).
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle.compact import compact_coefficients, stencil_start


def _fn(r):
    """f = exp(r/2) sin(3 r) and its exact derivatives up to order 4."""
    # derivatives of exp(a r) sin(b r): Im((a + i b)^k exp((a + i b) r))
    z = 0.5 + 3j
    return [np.imag(z ** k * np.exp(z * r)) for k in range(5)]


def _ops_exact(r):
    f = _fn(r)
    return {
        "d1": f[1],
        "d2": f[2],
        "d2s": f[2] + f[1] / r - f[0] / r**2,
        "d4s": f[4] + 2 * f[3] / r - 3 * f[2] / r**2 + 3 * f[1] / r**3 - 3 * f[0] / r**4,
    }, f[0]


def test_planar_uniform_limit_gives_classical_rationals():
    r = 1e7 + np.arange(11.0)  # h = 1, curvature 1e-7
    c, s = compact_coefficients(r)
    row = 5
    expect = {
        "d0": [Fraction(-1, 720), Fraction(124, 720), Fraction(474, 720), Fraction(124, 720), Fraction(-1, 720)],
        "d4s": [1, -4, 6, -4, 1],
        "d2": [Fraction(1, 12), Fraction(8, 12), Fraction(-18, 12), Fraction(8, 12), Fraction(1, 12)],
        "d2s": [Fraction(1, 12), Fraction(8, 12), Fraction(-18, 12), Fraction(8, 12), Fraction(1, 12)],
        "d1": [0, Fraction(-1, 2), 0, Fraction(1, 2), 0],
    }
    for fam, vals in expect.items():
        np.testing.assert_allclose(c[fam][row], [float(v) for v in vals], atol=2e-6)


def test_near_wall_rows_are_explicit():
    r = np.linspace(1.0, 2.0, 17)
    c, s = compact_coefficients(r)
    n = r.size
    for row in (0, 1, n - 2, n - 1):
        e = np.zeros(5)
        e[row - s[row]] = 1.0
        np.testing.assert_array_equal(c["d0"][row], e)
    assert list(s[:3]) == [0, 0, 0] and list(s[-3:]) == [n - 5] * 3
    assert list(stencil_start(9)) == [0, 0, 0, 1, 2, 3, 4, 4, 4]


def _trunc(n, stretch=1.5):
    xi = -1 + 2 * np.arange(n) / (n - 1)
    r = 1.0 + (1 + np.tanh(stretch * xi) / np.tanh(stretch)) / 2
    c, s = compact_coefficients(r)
    exact, f0 = _ops_exact(r)
    err = {}
    for fam in ("d1", "d2", "d2s", "d4s"):
        disc = sum(c[fam][:, j] * f0[s + j] for j in range(5))
        ref = sum(c["d0"][:, j] * exact[fam][s + j] for j in range(5))
        rows = slice(2, n - 2) if fam == "d4s" else slice(0, n)
        err[fam] = np.max(np.abs(disc - ref)[rows]) / np.max(np.abs(ref[rows]))
    return err


def test_truncation_order():
    e1, e2 = _trunc(33), _trunc(65)
    order = {k: np.log2(e1[k] / e2[k]) for k in e1}
    # the fourth-order operator reaches FP64 round-off (about eps * 16 / h^4
    # relative to the fourth derivative) near N_r = 33: measure it coarser
    order["d4s"] = np.log2(_trunc(13)["d4s"] / _trunc(25)["d4s"])
    # first derivative: fourth order on every row; second-order operators are
    # limited to third order by the one-sided near-wall rows; the fourth-order
    # operator is fifth order on centred rows
    assert order["d1"] > 3.6, order
    assert order["d2"] > 2.7 and order["d2s"] > 2.7, order
    assert order["d4s"] > 3.6, order


@pytest.mark.parametrize("fam,deg", [("d1", 4), ("d2", 4), ("d2s", 4), ("d4s", 4)])
def test_polynomial_exactness(fam, deg):
    """d_L p = d0 (L p) for polynomials of degree <= 4 on every row (the
    defining property), evaluated through an independent route: numpy's
    polynomial derivatives on the unscaled grid."""
    r = np.sort(np.random.default_rng(1).uniform(1.0, 2.0, 12))
    r[0], r[-1] = 1.0, 2.0
    c, s = compact_coefficients(r)
    coeffs = np.random.default_rng(2).standard_normal(deg + 1)
    P = np.polynomial.Polynomial(coeffs)
    d = [P.deriv(k)(r) if k else P(r) for k in range(5)]
    ops = {"d1": d[1], "d2": d[2], "d2s": d[2] + d[1] / r - d[0] / r**2,
           "d4s": d[4] + 2 * d[3] / r - 3 * d[2] / r**2 + 3 * d[1] / r**3 - 3 * d[0] / r**4}
    lhs = sum(c[fam][:, j] * d[0][s + j] for j in range(5))
    rhs = sum(c["d0"][:, j] * ops[fam][s + j] for j in range(5))
    scale = np.max(np.abs(c[fam])) * np.max(np.abs(d[0]))
    np.testing.assert_allclose(lhs, rhs, atol=1e-11 * scale)
