"""Fourth-order explicit compact finite-difference coefficients (oracle side).

Sec. 2.1 and the Appendix: radial derivatives use explicit compact schemes on
a stencil of 5 arbitrarily spaced points, with coefficients found by matching
the discrete derivative of known functions (polynomials) to the analytic one.
"Explicit" (in the sense of Thomas, 1953) means that every operator shares one
"denominator" stencil d0: an operator term L(g) at row n is read as
sum_j dL[n, j] g(r_{sigma_n + j}) and stands for sum_j d0[n, j] (L g)(r_{sigma_n + j}),
so every discrete equation row is the continuous equation multiplied by d0.

Five operator families (Appendix; the fourth-order one has its own set because
D D_* D D_* contains a third derivative):

    d0   identity (the shared denominator)
    d1   D            f'
    d2   D D          f''
    d2s  D D_*        f'' + f'/r - f/r^2
    d4s  D D_* D D_*  f'''' + 2 f'''/r - 3 f''/r^2 + 3 f'/r^3 - 3 f/r^4

Readings (the paper refers to another report for the full construction):

* Stencil of row n: points sigma_n .. sigma_n + 4 with
  sigma_n = clamp(n - 2, 0, N_r - 5).
* Centred rows (sigma_n = n - 2): d0 and d4s together are fixed by exactness
  of d4s f = d0 (D D_* D D_* f) on the monomials of degree 0..8, plus the
  normalisation sum(d0) = 1 (10 equations, 10 unknowns).
* The four near-wall rows 0, 1, N_r - 2, N_r - 1: d0 = e_n (one-sided explicit
  formulas); d4s then follows from degree 0..4 exactness.
* For every row, d1, d2 and d2s follow from exactness on degrees 0..4 given d0.

Monomials are written in the local variable x = (r - r_n) / h_n with
h_n = (r_{sigma+4} - r_sigma) / 4, and the operators are scaled by h_n^k, so
every linear system has O(1) entries; the returned coefficients are in
physical units.
"""

from math import factorial

import numpy as np

FAMILIES = ("d0", "d1", "d2", "d2s", "d4s")


def stencil_start(nr):
    """sigma_n = clamp(n - 2, 0, N_r - 5) for n = 0..N_r-1."""
    n = np.arange(nr)
    return np.clip(n - 2, 0, nr - 5)


def _deriv_monomial(x, p, k):
    """h^k d^k/dr^k of x^p, where x = (r - r_n)/h, evaluated at x."""
    if k > p:
        return np.zeros_like(x)
    return factorial(p) / factorial(p - k) * x ** (p - k)


def _scaled_operator(name, x, p, q):
    """h^k (L x^p) at points x for operator family `name`; q = h / r there."""
    dk = [_deriv_monomial(x, p, k) for k in range(5)]
    if name == "d1":
        return dk[1]
    if name == "d2":
        return dk[2]
    if name == "d2s":
        return dk[2] + q * dk[1] - q * q * dk[0]
    if name == "d4s":
        return dk[4] + 2 * q * dk[3] - 3 * q**2 * dk[2] + 3 * q**3 * dk[1] - 3 * q**4 * dk[0]
    raise KeyError(name)


ORDER = {"d1": 1, "d2": 2, "d2s": 2, "d4s": 4}


def compact_coefficients(r):
    """Return ({family: (N_r, 5) array}, sigma) for the radial grid r.

    Follows Sec. 2.1 and the Appendix with the readings listed in the module
    docstring.
    """
    r = np.asarray(r, dtype=np.float64)
    nr = r.size
    if nr < 7:
        raise ValueError("need at least 7 radial points")
    sigma = stencil_start(nr)
    out = {f: np.zeros((nr, 5)) for f in FAMILIES}
    for n in range(nr):
        s = sigma[n]
        pts = r[s:s + 5]
        h = (pts[4] - pts[0]) / 4.0
        x = (pts - r[n]) / h
        q = h / pts
        vander = np.array([x ** p for p in range(5)])  # (p, j)
        centred = (s == n - 2)
        if centred:
            # unknowns: d0[0..4], e[0..4] with e = h^4 d4s
            a = np.zeros((10, 10))
            b = np.zeros(10)
            for p in range(9):
                a[p, 5:] = x ** p
                a[p, :5] = -_scaled_operator("d4s", x, p, q)
            a[9, :5] = 1.0
            b[9] = 1.0
            sol = np.linalg.solve(a, b)
            d0 = sol[:5]
            out["d4s"][n] = sol[5:] / h ** 4
        else:
            d0 = np.zeros(5)
            d0[n - s] = 1.0
            rhs = np.array([
                np.dot(d0, _scaled_operator("d4s", x, p, q)) for p in range(5)
            ])
            out["d4s"][n] = np.linalg.solve(vander, rhs) / h ** 4
        out["d0"][n] = d0
        for fam in ("d1", "d2", "d2s"):
            rhs = np.array([np.dot(d0, _scaled_operator(fam, x, p, q)) for p in range(5)])
            out[fam][n] = np.linalg.solve(vander, rhs) / h ** ORDER[fam]
    return out, sigma


def apply(coef, sigma, g):
    """(d_L g)_n = sum_j coef[n, j] g[sigma_n + j]; g has r as its first axis."""
    g = np.asarray(g)
    shape = (coef.shape[0],) + (1,) * (g.ndim - 1)
    out = np.zeros(g.shape, dtype=np.result_type(g, np.float64))
    for j in range(5):
        out += coef[:, j].reshape(shape) * g[sigma + j]
    return out
