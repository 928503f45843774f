"""Closed-form targets for the oracle pins, built from the primitive-variable
Navier--Stokes equations in cylindrical coordinates (not from the paper's
rewritten equations).

For one Fourier mode exp(i (m theta + alpha z)) with velocity (u, v, w) =
(axial, radial, azimuthal) components and products UU..WW:

    vector Laplacian:  Vu = u'' + u'/r - k^2 u
                       Vv = v'' + v'/r - k^2 v - v/r^2 - 2 i m w / r^2
                       Vw = w'' + w'/r - k^2 w - w/r^2 + 2 i m v / r^2
    advection (conservative form, with the centrifugal and Coriolis terms):
                       HU = -(i alpha UU + (r UV)'/r + i m UW / r)
                       HV = -(i alpha UV + (r VV)'/r + i m VW / r - WW / r)
                       HW = -(i alpha UW + (r^2 VW)'/r^2 + i m WW / r)

Eliminating the pressure with i alpha (u-eq) + (i m / r)(w-eq) and continuity
D_* v = -(i alpha u + i m w / r) gives, for any forcing (Fu, Fv, Fw),

    d/dt [v - D(a D_* v)] = D[a (i alpha Fu + (i m / r) Fw)] + Fv,
    d/dt eta              = (i m / r) Fu - i alpha Fw,

with a = 1 / k^2 and eta = (i m / r) u - i alpha w.
"""

import numpy as np
import sympy as sp

r = sp.Symbol("r", positive=True)


def _lam(expr):
    f = sp.lambdify(r, expr, "numpy")

    def call(x):
        return np.asarray(f(np.asarray(x, dtype=np.float64)), dtype=np.complex128) * np.ones_like(x)
    return call


class Mode:
    """Manufactured smooth fields on one mode and their exact operators."""

    def __init__(self, ri, ro, alpha, m):
        d = ro - ri
        x = (2 * r - ri - ro) / d
        al, mm = sp.nsimplify(alpha), sp.nsimplify(m)
        I = sp.I
        k2 = al**2 + mm**2 / r**2
        a = 1 / k2
        D = lambda f: sp.diff(f, r)
        Ds = lambda f: sp.diff(f, r) + f / r
        v = (1 - x**2) ** 2 * (1 + sp.Rational(3, 10) * x + sp.Rational(1, 5) * I * x**2)
        eta = (1 - x**2) * (sp.Rational(1, 2) + sp.Rational(7, 10) * I * x + sp.Rational(1, 5) * x**3)
        dsv = Ds(v)
        u = a * (I * al * dsv - I * mm / r * eta)
        w = a * (I * mm / r * dsv + I * al * eta)
        prods = {
            "uu": sp.cos(r) + I * r / 3,
            "uv": (1 - x**2) * sp.exp(r / 3),
            "uw": sp.sin(2 * r) - I * sp.cos(r / 2),
            "vv": (1 - x**2) ** 2 * (1 + x),
            "vw": (1 - x**2) * (sp.Rational(1, 2) - I * x**2),
            "ww": 1 + x**2 + I * sp.sin(r),
        }
        UU, UV, UW, VV, VW, WW = (prods[k] for k in ("uu", "uv", "uw", "vv", "vw", "ww"))
        Vu = D(D(u)) + D(u) / r - k2 * u
        Vv = D(D(v)) + D(v) / r - k2 * v - v / r**2 - 2 * I * mm * w / r**2
        Vw = D(D(w)) + D(w) / r - k2 * w - w / r**2 + 2 * I * mm * v / r**2
        HU = -(I * al * UU + D(r * UV) / r + I * mm * UW / r)
        HV = -(I * al * UV + D(r * VV) / r + I * mm * VW / r - WW / r)
        HW = -(I * al * UW + D(r**2 * VW) / r**2 + I * mm * WW / r)
        self.fields = {"v": v, "eta": eta, "u": u, "w": w, "dv": D(v),
                       "c": I * al * u + I * mm / r * w, **prods}
        self.targets = {
            "v_mass": v - D(a * dsv),
            "v_visc": D(a * (I * al * Vu + I * mm / r * Vw)) + Vv,
            "v_nl": D(a * (I * al * HU + I * mm / r * HW)) + HV,
            "eta_visc": I * mm / r * Vu - I * al * Vw,
            "eta_nl": I * mm / r * HU - I * al * HW,
        }
        self.f = {k: _lam(e) for k, e in self.fields.items()}
        self.t = {k: _lam(sp.simplify(e) if k.endswith("mass") else e) for k, e in self.targets.items()}
        self.alpha = alpha
        self.m = m


class MeanProfiles:
    """Manufactured mean profiles and the exact mean-flow operators:
    axial  D_* D u  and forcing -(UV)' - UV/r;
    azimuthal  D_* D w - w/r^2  and forcing -(VW)' - 2 VW/r."""

    def __init__(self, ri, ro):
        d = ro - ri
        x = (2 * r - ri - ro) / d
        D = lambda f: sp.diff(f, r)
        um = (1 - x**2) * (1 + x / 2) * sp.exp(r / 4)
        wm = sp.cos(r) + r**2 / 7
        uv = sp.sin(r) * (1 + x**2)
        vw = sp.exp(-r) * (1 - x**2)
        self.f = {k: _lam(e) for k, e in {"u": um, "w": wm, "uv": uv, "vw": vw}.items()}
        self.t = {k: _lam(e) for k, e in {
            "u_visc": D(D(um)) + D(um) / r,
            "w_visc": D(D(wm)) + D(wm) / r - wm / r**2,
            "u_nl": -(D(uv) + uv / r),
            "w_nl": -(D(vw) + 2 * vw / r),
        }.items()}
