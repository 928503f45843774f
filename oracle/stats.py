"""Torque, wall shear, friction Reynolds number and kinetic energy (oracle).

Torque, eq. (torque) of Sec. 3: the printed formula places the absolute value
around dw/dr only, which would give 4.19 for the laminar case at zeta = 0.5
while Table 2 prints 16.7551 = 4 pi / (1 - zeta^2).  The reading taken is
g = |D w - w / r| at the wall, i.e. the r-theta shear, with D w from the
explicit one-sided compact rows at the walls, and

    T_i = 2 pi R_i g_i,   T_o = 2 pi R_o^2 g_o / R_i,

the torques per unit length made non-dimensional with mu W_i R_i.

Sec. 5: tau_w = nu g at each wall, u_tau = sqrt(tau_w), and
Re_tau = u_tau delta / nu with delta = h = d / 2 (half the gap).

Kinetic energy: E = sum_n w_n r_n sum_{j,l} c_j (|u|^2 + |v|^2 + |w|^2)
/ (2 sum_n w_n r_n) with trapezoidal weights w_n and c_0 = 1, c_{j>0} = 2
(Parseval over the stored half spectrum).  ``energy`` includes the mean flow,
``energy_pert`` excludes the (0,0) mode.

Radial profiles (Sec. 5: mean azimuthal velocity and the variances of the
velocity fluctuations across the gap): at each radial node, averages over
theta and z.  The mean profiles are the (0,0) mode; the fluctuation of f is
f minus its plane mean, so its variance is, by Parseval over the stored half
spectrum, <f'f'>(r) = sum_{(j,l) != (0,0)} c_j |f_hat(r, j, l)|^2, and the
covariance <v'w'>(r) = sum c_j Re(v_hat conj(w_hat)).
"""

import numpy as np


def trapezoid_weights(r):
    w = np.zeros_like(r)
    w[1:-1] = 0.5 * (r[2:] - r[:-2])
    w[0] = 0.5 * (r[1] - r[0])
    w[-1] = 0.5 * (r[-1] - r[-2])
    return w


def wall_shear(ops, r, w_mean):
    d1 = ops.coef["d1"]
    nr = r.size
    dw_in = np.dot(d1[0], w_mean[0:5])
    dw_out = np.dot(d1[nr - 1], w_mean[nr - 5:nr])
    g_in = abs(dw_in - w_mean[0] / r[0])
    g_out = abs(dw_out - w_mean[nr - 1] / r[nr - 1])
    return g_in, g_out


def statistics(orc, u, w):
    d = orc.disc
    r = d.r
    g_in, g_out = wall_shear(orc.ops, r, orc.w_mean)
    tau_in, tau_out = d.nu * g_in, d.nu * g_out
    half_gap = 0.5 * orc.geo.gap
    cj = np.where(np.arange(d.nj) == 0, 1.0, 2.0)
    cflat = np.repeat(cj, d.nl)
    dens = (np.abs(u) ** 2 + np.abs(orc.v) ** 2 + np.abs(w) ** 2) * cflat[None, :]
    per_r = dens.sum(axis=1)
    # the perturbation sum is taken over the other modes directly (subtracting
    # the O(1) mean-flow term from the total would cancel catastrophically)
    pert = np.ones(dens.shape[1], dtype=bool)
    pert[orc.mean_index] = False
    per_r_pert = dens[:, pert].sum(axis=1)
    wr = trapezoid_weights(r) * r
    vol = wr.sum()
    finite = (np.all(np.isfinite(orc.v)) and np.all(np.isfinite(orc.eta))
              and np.all(np.isfinite(orc.u_mean)) and np.all(np.isfinite(orc.w_mean)))
    return {
        "time": orc.time,
        "torque_in": 2 * np.pi * d.ri * g_in,
        "torque_out": 2 * np.pi * d.ro ** 2 * g_out / d.ri,
        "tau_in": tau_in,
        "tau_out": tau_out,
        "retau_in": np.sqrt(tau_in) * half_gap / d.nu,
        "retau_out": np.sqrt(tau_out) * half_gap / d.nu,
        "energy": float(np.dot(wr, per_r) / (2 * vol)),
        "energy_pert": float(np.dot(wr, per_r_pert) / (2 * vol)),
        "steps": orc.steps,
        "nonfinite": int(not finite),
    }


def plane_profiles(orc, u, w):
    """Mean profiles and fluctuation (co)variances at every radial node, from
    the spectral velocities u, w (mean in the (0,0) slot) and orc.v.  Returns
    a dict of arrays of length N_r: u_mean, w_mean, uu, vv, ww, vw."""
    d = orc.disc
    cj = np.where(np.arange(d.nj) == 0, 1.0, 2.0)
    c = np.repeat(cj, d.nl)[None, :].copy()
    c[0, orc.mean_index] = 0.0  # fluctuations: the plane mean is left out
    v = orc.v
    return {
        "u_mean": orc.u_mean.copy(),
        "w_mean": orc.w_mean.copy(),
        "uu": (c * np.abs(u) ** 2).sum(axis=1),
        "vv": (c * np.abs(v) ** 2).sum(axis=1),
        "ww": (c * np.abs(w) ** 2).sum(axis=1),
        "vw": (c * (v * np.conj(w)).real).sum(axis=1),
    }
