"""Pins of the oracle's statistics: kinetic energy against closed-form
integrals, the wall-shear reading of eq. (torque) against the exact Couette
shear, and the input generator's amplitude recipe."""

import numpy as np
from scipy.integrate import quad

from oracle import Geometry, Oracle
from paper_0711_1429_amd.synth import initial_fields, couette_profile
from tests.analytic import Mode


def test_mean_flow_energy_is_the_volume_average():
    zeta = 0.6
    orc = Oracle(Geometry(zeta=zeta, re=100.0, nr=129, ntheta=8, nz=8, dt=1e-3, stretch=1.0))
    r = orc.disc.r
    w = couette_profile(r, zeta, 1.0, 0.3)
    orc.w_mean = w
    ri, ro = orc.disc.ri, orc.disc.ro
    a = (0.3 * ro - ri) / (ro**2 - ri**2)
    b = ri - a * ri**2
    num = quad(lambda x: x * (a * x + b / x) ** 2, ri, ro)[0]
    den = 0.5 * (ro**2 - ri**2)
    s = orc.stats()
    assert abs(s["energy"] / (num / (2 * den)) - 1) < 1e-4
    assert s["energy_pert"] == 0.0


def test_perturbation_energy_of_one_mode():
    """A single (j=1, l=2) mode: E = c_1 int r (|u|^2+|v|^2+|w|^2) dr / (2 int r dr)
    with c_1 = 2 and u, w from continuity (closed form)."""
    orc = Oracle(Geometry(zeta=0.5, re=100.0, nr=129, ntheta=8, nz=8, dt=1e-3, lz=2.0))
    j, l = 1, 2
    kz = orc.disc.kz
    mode = Mode(orc.disc.ri, orc.disc.ro, orc.disc.alpha[l + kz], orc.disc.m[j])
    r = orc.disc.r
    v = np.zeros((r.size, orc.disc.nj, orc.disc.nl), dtype=complex)
    e = np.zeros_like(v)
    v[:, j, l + kz] = mode.f["v"](r)
    e[:, j, l + kz] = mode.f["eta"](r)
    orc.load(v, e, np.zeros(r.size), np.zeros(r.size))
    dens = lambda x: x * sum(abs(mode.f[k](np.array([x]))[0]) ** 2 for k in ("u", "v", "w"))
    ri, ro = orc.disc.ri, orc.disc.ro
    ref = 2 * quad(dens, ri, ro, limit=200)[0] / (2 * 0.5 * (ro**2 - ri**2))
    s = orc.stats()
    assert abs(s["energy_pert"] / ref - 1) < 1e-4, (s["energy_pert"], ref)


def test_torque_reading_on_exact_couette_profiles():
    """g = |D w - w/r| at the walls of w = A r + B/r is 2|B|/r^2, so
    T_i = 4 pi |B| / R_i and T_o = 2 pi R_o^2 (2|B|/R_o^2) / R_i = T_i."""
    for zeta, wo in ((0.5, 0.0), (0.883, 0.0), (0.7, -0.4)):
        orc = Oracle(Geometry(zeta=zeta, re=100.0, nr=97, ntheta=8, nz=8, dt=1e-3))
        r = orc.disc.r
        orc.w_mean = couette_profile(r, zeta, 1.0, wo)
        ri, ro = orc.disc.ri, orc.disc.ro
        a = (wo * ro - ri) / (ro**2 - ri**2)
        b = ri - a * ri**2
        s = orc.stats()
        assert abs(s["torque_in"] / (4 * np.pi * abs(b) / ri) - 1) < 1e-6
        assert abs(s["torque_out"] / (4 * np.pi * abs(b) / ri) - 1) < 1e-6


def test_generator_amplitude_is_the_rms_radial_velocity():
    """Volume RMS of v' from the generated fields (trapezoid on a fine grid)
    equals the requested amplitude; phases are reproducible per seed."""
    zeta, nt, nz = 0.883, 16, 12
    r = np.linspace(zeta / (1 - zeta), 1 / (1 - zeta), 401)
    v, e, um, wm = initial_fields(r, zeta, nt, nz, 0.05, seed=3)
    cj = np.where(np.arange(v.shape[1]) == 0, 1.0, 2.0)[None, :, None]
    dens = np.sum(cj * np.abs(v) ** 2, axis=(1, 2))
    rms = np.sqrt(np.trapezoid(r * dens, r) / np.trapezoid(r, r))
    assert abs(rms / 0.05 - 1) < 1e-4
    v2 = initial_fields(r, zeta, nt, nz, 0.05, seed=3)[0]
    assert np.array_equal(v, v2)
    kz = (v.shape[2] - 1) // 2
    np.testing.assert_array_equal(v[:, 0, kz - 1], np.conj(v[:, 0, kz + 1]))
    assert np.all(v[:, 0, kz] == 0)
    assert wm[0] == 1.0 and wm[-1] == 0.0
