"""Seeded synthetic inputs for the Taylor--Couette substep.

This module is the only code shared by the HIP library's callers and the
test oracle.  It draws random numbers and samples closed-form profiles; it
holds none of the method's arithmetic (no compact operators, no transforms, no
recovery, no time stepping).

Initial condition (Sec. 4, "Computational procedures"): the laminar
circular-Couette profile plus divergence-free disturbances of random phase on
the whole set of retained Fourier modes.  Recipe:

* base flow: mean azimuthal velocity w(r) = A r + B / r through w(R_i) = 1 and
  w(R_o) = W_o (eq. (laminar-solution) when W_o = 0), mean axial velocity 0;
* every stored mode (j, l) != (0, 0), with j = 0 only for l > 0 (its l < 0
  mirror is the complex conjugate): v = P exp(i phi1) (1 - x^2)^2 and
  eta = (P / d) exp(i phi2) (1 - x^2), x = (2 r - R_i - R_o) / d.  Both
  vanish at the walls together with dv/dr, so the no-slip conditions hold and
  the velocity recovered through continuity is divergence free;
* phases phi1, phi2 ~ U[0, 2 pi) from numpy's default_rng(seed), drawn mode by
  mode in j-major, l-ascending order, phi1 before phi2;
* one flat amplitude P for all modes, chosen so that the volume RMS of the
  radial velocity perturbation equals ``amplitude``.  In closed form,
  <v'^2>_V = P^2 C (128 / 315) with C = sum over stored modes of c_j
  (c_0 = 1, c_{j>0} = 2), since int r (1 - x^2)^4 dr / int r dr = 128/315.
"""

import numpy as np


def geometry_radii(zeta, gap):
    return gap * zeta / (1.0 - zeta), gap / (1.0 - zeta)


def couette_profile(r, zeta, gap, w_outer):
    """Laminar azimuthal velocity A r + B / r with w(R_i) = 1, w(R_o) = W_o."""
    ri, ro = geometry_radii(zeta, gap)
    a = (w_outer * ro - ri) / (ro * ro - ri * ri)
    b = ri - a * ri * ri
    w = a * r + b / r
    w = np.array(w, dtype=np.float64)
    w[0] = 1.0
    w[-1] = w_outer
    return w


def initial_fields(r, zeta, ntheta, nz, amplitude, seed, gap=1.0, w_outer=0.0):
    """Return (v_hat, eta_hat, u_mean, w_mean).

    v_hat and eta_hat are complex128 arrays of shape (N_r, K_theta + 1, 2 K_z + 1)
    laid out [r][j][l + K_z]; u_mean and w_mean are float64 of shape (N_r,).
    """
    r = np.asarray(r, dtype=np.float64)
    nr = r.size
    kt = (ntheta - 1) // 3
    kz = (nz - 1) // 3
    nj, nl = kt + 1, 2 * kz + 1
    ri, ro = geometry_radii(zeta, gap)
    x = (2.0 * r - ri - ro) / gap
    pv = (1.0 - x * x) ** 2
    pe = (1.0 - x * x) / gap
    pv[0] = pv[-1] = 0.0
    pe[0] = pe[-1] = 0.0

    drawn = [(j, l) for j in range(nj) for l in range(-kz, kz + 1) if j > 0 or l > 0]
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=(len(drawn), 2))
    count = 2 * kz + 2 * kt * nl  # sum of c_j over stored modes other than (0,0)
    p = amplitude / np.sqrt(count * 128.0 / 315.0) if count > 0 else 0.0

    v = np.zeros((nr, nj, nl), dtype=np.complex128)
    eta = np.zeros((nr, nj, nl), dtype=np.complex128)
    for (j, l), (f1, f2) in zip(drawn, phases):
        c1 = p * np.exp(1j * f1)
        c2 = p * np.exp(1j * f2)
        v[:, j, l + kz] = c1 * pv
        eta[:, j, l + kz] = c2 * pe
        if j == 0:
            v[:, 0, -l + kz] = np.conj(c1) * pv
            eta[:, 0, -l + kz] = np.conj(c2) * pe
    u_mean = np.zeros(nr)
    w_mean = couette_profile(r, zeta, gap, w_outer)
    return v, eta, u_mean, w_mean


# Workloads: the sizes of the paper's validation and turbulent cases as used
# by the tests and the benchmark.  zeta = 0.883 is the paper's small-gap
# geometry (Sec. 4); "pert" is the RMS radial-velocity amplitude.
WORKLOADS = {
    "tc-small-fp64": dict(zeta=0.883, re=150.0, nr=33, ntheta=32, nz=32, dt=1e-3,
                          stretch=0.0, amplitude=1e-3, seed=0, steps=10),
    "tc-medium-fp64": dict(zeta=0.883, re=2000.0, nr=65, ntheta=128, nz=128, dt=5e-4,
                           stretch=0.0, amplitude=0.05, seed=1, steps=200),
    "tc-turbulent-fp64": dict(zeta=0.883, re=8000.0, nr=129, ntheta=768, nz=384, dt=2e-4,
                              stretch=1.5, amplitude=0.1, seed=2, steps=1000),
}


def batched_instances(n=64, seed=4):
    """The batched workload: n independent instances with radius ratio
    ~ U[0.70, 0.98], Re ~ U[500, 4000], N_r in {33, 49, 65} and
    (N_theta, N_z) in {64x64, 96x64, 128x128}, each drawn uniformly and
    independently from default_rng(seed) in that order (all radius ratios,
    then all Re, then all N_r choices, then all shape choices); instance b
    uses perturbation seed 4000 + b, amplitude 1e-2, dt = 5e-4."""
    rng = np.random.default_rng(seed)
    zeta = rng.uniform(0.70, 0.98, n)
    re = rng.uniform(500.0, 4000.0, n)
    nr = rng.choice(np.array([33, 49, 65]), n)
    shapes = [(64, 64), (96, 64), (128, 128)]
    sh = rng.integers(0, 3, n)
    out = []
    for b in range(n):
        nt, nz = shapes[int(sh[b])]
        out.append(dict(zeta=float(zeta[b]), re=float(re[b]), nr=int(nr[b]), ntheta=nt, nz=nz, dt=5e-4,
                        stretch=0.0, amplitude=1e-2, seed=4000 + b, steps=100))
    return out
