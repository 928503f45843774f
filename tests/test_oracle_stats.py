"""Pins of the oracle's statistics: kinetic energy against closed-form
integrals, the wall-shear reading of eq. (torque) against the exact Couette
shear, the radial profiles of the fluctuation variances against plane
averages taken in physical space, and the input generator's amplitude
recipe."""

import numpy as np
from scipy.integrate import quad

from oracle import Geometry, Oracle
from oracle.spectral import to_physical
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


def test_profiles_are_plane_averages_in_physical_space():
    """<f'f'>(r) and <v'w'>(r) from the Parseval sums equal the averages over
    the theta-z plane of the physical fluctuations (each field minus its plane
    mean), computed on the transform grid; the mean profiles are the (0,0)
    mode."""
    g = Geometry(zeta=0.7, re=300.0, nr=17, ntheta=24, nz=20, dt=1e-3, stretch=1.0)
    orc = Oracle(g)
    v, e, um, wm = initial_fields(orc.disc.r, g.zeta, g.ntheta, g.nz, 0.05, seed=11)
    orc.load(v, e, um, wm)
    prof = orc.profiles()
    dv, u, w, c = orc.velocity()
    shape = (g.nr, orc.disc.nj, orc.disc.nl)
    phys = {k: to_physical(a.reshape(shape), g.ntheta, g.nz) for k, a in (("u", u), ("v", orc.v), ("w", w))}
    fl = {k: f - f.mean(axis=(1, 2), keepdims=True) for k, f in phys.items()}
    np.testing.assert_allclose(phys["w"].mean(axis=(1, 2)), prof["w_mean"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(phys["u"].mean(axis=(1, 2)), prof["u_mean"], rtol=0, atol=1e-13)
    for key, a, b in (("uu", "u", "u"), ("vv", "v", "v"), ("ww", "w", "w"), ("vw", "v", "w")):
        ref = (fl[a] * fl[b]).mean(axis=(1, 2))
        scale = np.abs(ref).max()
        assert scale > 1e-6
        np.testing.assert_allclose(prof[key], ref, rtol=0, atol=1e-12 * scale)
    # no-slip walls: every fluctuation vanishes there
    for key in ("uu", "vv", "ww", "vw"):
        assert abs(prof[key][0]) < 1e-20 and abs(prof[key][-1]) < 1e-20


def test_profile_of_one_mode_is_twice_its_squared_amplitude():
    """A single (j=1, l=2) mode f = a exp(i(m theta + alpha z)) + c.c. has
    plane variance 2 |a|^2 at every radius; here for v, whose amplitude is the
    closed-form eigenfunction."""
    orc = Oracle(Geometry(zeta=0.5, re=100.0, nr=33, ntheta=8, nz=8, dt=1e-3, lz=2.0))
    j, l = 1, 2
    kz = orc.disc.kz
    mode = Mode(orc.disc.ri, orc.disc.ro, orc.disc.alpha[l + kz], orc.disc.m[j])
    r = orc.disc.r
    v = np.zeros((r.size, orc.disc.nj, orc.disc.nl), dtype=complex)
    e = np.zeros_like(v)
    v[:, j, l + kz] = mode.f["v"](r)
    e[:, j, l + kz] = mode.f["eta"](r)
    orc.load(v, e, np.zeros(r.size), np.zeros(r.size))
    prof = orc.profiles()
    np.testing.assert_allclose(prof["vv"], 2 * np.abs(mode.f["v"](r)) ** 2, rtol=1e-13, atol=1e-30)
