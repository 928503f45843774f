"""Pins of the oracle's Fourier transforms and dealiased products: direct DFT
sums and direct convolutions on tiny grids (brute force), round trip and
Parseval."""

import numpy as np

from oracle.spectral import to_physical, to_spectral, products


def _random_spectrum(rng, nr, nj, nl):
    kz = (nl - 1) // 2
    f = rng.standard_normal((nr, nj, nl)) + 1j * rng.standard_normal((nr, nj, nl))
    # j = 0 column Hermitian: f[0, -l] = conj f[0, l], f[0, 0] real
    for l in range(1, kz + 1):
        f[:, 0, kz - l] = np.conj(f[:, 0, kz + l])
    f[:, 0, kz] = f[:, 0, kz].real
    return f


def _direct_physical(fhat, nt, nz):
    nr, nj, nl = fhat.shape
    kz = (nl - 1) // 2
    out = np.zeros((nr, nz, nt))
    for q in range(nz):
        for p in range(nt):
            s = np.zeros(nr, dtype=complex)
            for j in range(-(nj - 1), nj):
                for l in range(-kz, kz + 1):
                    c = fhat[:, j, l + kz] if j >= 0 else np.conj(fhat[:, -j, -l + kz])
                    s += c * np.exp(2j * np.pi * (j * p / nt + l * q / nz))
            assert np.max(np.abs(s.imag)) < 1e-12
            out[:, q, p] = s.real
    return out


def test_inverse_transform_is_the_fourier_sum():
    rng = np.random.default_rng(0)
    nt, nz = 8, 7
    nj, nl = (nt - 1) // 3 + 1, 2 * ((nz - 1) // 3) + 1
    f = _random_spectrum(rng, 2, nj, nl)
    np.testing.assert_allclose(to_physical(f, nt, nz), _direct_physical(f, nt, nz), atol=1e-12)


def test_forward_transform_is_the_normalised_dft():
    rng = np.random.default_rng(1)
    nt, nz = 10, 8
    phys = rng.standard_normal((2, nz, nt))
    nj, nl = (nt - 1) // 3 + 1, 2 * ((nz - 1) // 3) + 1
    kz = (nl - 1) // 2
    got = to_spectral(phys, nj, nl)
    for j in range(nj):
        for l in range(-kz, kz + 1):
            ref = np.zeros(2, dtype=complex)
            for q in range(nz):
                for p in range(nt):
                    ref += phys[:, q, p] * np.exp(-2j * np.pi * (j * p / nt + l * q / nz))
            np.testing.assert_allclose(got[:, j, l + kz], ref / (nt * nz), atol=1e-13)


def test_round_trip_and_parseval():
    rng = np.random.default_rng(2)
    nt, nz = 24, 12
    nj, nl = (nt - 1) // 3 + 1, 2 * ((nz - 1) // 3) + 1
    f = _random_spectrum(rng, 3, nj, nl)
    phys = to_physical(f, nt, nz)
    np.testing.assert_allclose(to_spectral(phys, nj, nl), f, atol=1e-13)
    cj = np.where(np.arange(nj) == 0, 1.0, 2.0)[None, :, None]
    np.testing.assert_allclose(np.mean(phys ** 2, axis=(1, 2)), np.sum(cj * np.abs(f) ** 2, axis=(1, 2)), rtol=1e-12)


def test_dealiased_product_equals_truncated_convolution():
    """With K = floor((N-1)/3) the pseudo-spectral product of two band-limited
    fields equals their exact convolution truncated to |j| <= K_theta,
    |l| <= K_z: no aliasing survives (the 3/2 rule)."""
    rng = np.random.default_rng(3)
    nt, nz = 12, 9
    nj, nl = (nt - 1) // 3 + 1, 2 * ((nz - 1) // 3) + 1
    kt, kz = nj - 1, (nl - 1) // 2
    a = _random_spectrum(rng, 1, nj, nl)
    b = _random_spectrum(rng, 1, nj, nl)
    zero = np.zeros_like(a)
    P = products(a, b, zero, nt, nz)  # u = a, v = b, w = 0 -> uv = a b

    def full(c, j, l):
        if abs(j) > kt or abs(l) > kz:
            return 0.0
        return c[0, j, l + kz] if j >= 0 else np.conj(c[0, -j, -l + kz])

    for j in range(nj):
        for l in range(-kz, kz + 1):
            s = 0.0
            for j1 in range(-kt, kt + 1):
                for l1 in range(-kz, kz + 1):
                    s += full(a, j1, l1) * full(b, j - j1, l - l1)
            np.testing.assert_allclose(P["uv"][0, j, l + kz], s, atol=1e-12)
