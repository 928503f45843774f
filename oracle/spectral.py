"""Fourier transforms and dealiased products (oracle side).

Appendix: theta and z are homogeneous and expanded in Fourier series; the
nonlinear terms HU, HV, HW are evaluated pseudo-spectrally from the six
products uu, uv, uw, vv, vw, ww of the physical velocities.

Convention (reading; the paper prints none): with theta_p = p Theta / N_theta
and z_q = q L_z / N_z,

    f_hat[j, l] = 1/(N_theta N_z) sum_{p,q} f[p, q] exp(-i (m_j theta_p + alpha_l z_q))
    f[p, q]     = sum_{j,l} f_hat[j, l] exp(+i (m_j theta_p + alpha_l z_q)),

so m_j theta_p = 2 pi j p / N_theta and alpha_l z_q = 2 pi l q / N_z.  Spectral
arrays hold j = 0..K_theta and l = -K_z..K_z at index l + K_z, shape
(N_r, nj, nl); negative j follow from f_hat[-j, -l] = conj(f_hat[j, l]).
Truncating the forward transform to |j| <= K_theta, |l| <= K_z with
K = floor((N - 1)/3) removes every alias of a quadratic product (3/2 rule).

The transforms use numpy's pocketfft (a library FFT as a step); the brute-force
tests compare them with direct DFT sums.
"""

import numpy as np


def to_physical(fhat, ntheta, nz):
    """Spectral (N_r, nj, nl) -> physical (N_r, N_z, N_theta), real."""
    nr, nj, nl = fhat.shape
    kz = (nl - 1) // 2
    full = np.zeros((nr, nz, ntheta // 2 + 1), dtype=np.complex128)
    for li in range(nl):
        l = li - kz
        full[:, l % nz, :nj] = fhat[:, :, li]
    # inverse transform without normalisation: irfftn(norm="forward") applies none
    return np.fft.irfftn(full, s=(nz, ntheta), axes=(1, 2), norm="forward")


def to_spectral(f, nj, nl):
    """Physical (N_r, N_z, N_theta) -> truncated spectral (N_r, nj, nl),
    including the 1/(N_theta N_z) normalisation."""
    nr, nz, ntheta = f.shape
    kz = (nl - 1) // 2
    full = np.fft.rfftn(f, axes=(1, 2), norm="forward")
    out = np.empty((nr, nj, nl), dtype=np.complex128)
    for li in range(nl):
        l = li - kz
        out[:, :, li] = full[:, l % nz, :nj]
    return out


PRODUCTS = ("uu", "uv", "uw", "vv", "vw", "ww")


def products(u_hat, v_hat, w_hat, ntheta, nz):
    """Dealiased Fourier coefficients of the six velocity products
    (Appendix, the terms uu..ww of eq. (final-v) and eq. (final-eta))."""
    nj, nl = u_hat.shape[1:]
    u = to_physical(u_hat, ntheta, nz)
    v = to_physical(v_hat, ntheta, nz)
    w = to_physical(w_hat, ntheta, nz)
    phys = {"uu": u * u, "uv": u * v, "uw": u * w, "vv": v * v, "vw": v * w, "ww": w * w}
    return {k: to_spectral(phys[k], nj, nl) for k in PRODUCTS}
