"""Pins for box 1 of Fig. 1: the normalised Gaussian (Eq. 7), the periodic
convolution (Eq. 6) and the partially coherent modulus constraint."""

import math

import numpy as np
import pytest

import oracle as ora


def test_kernel_normalised_and_oriented():
    g = ora.gaussian_kernel(1.3, 0.7, 11)
    assert g.shape == (11, 11)
    assert abs(g.sum() - 1.0) < 1e-15
    h = 5
    # sigma1 acts along x (columns), sigma2 along y (rows): Eq. (7)
    assert abs(g[h, h + 1] / g[h, h] - math.exp(-1 / (2 * 1.3 ** 2))) < 1e-14
    assert abs(g[h + 1, h] / g[h, h] - math.exp(-1 / (2 * 0.7 ** 2))) < 1e-14
    assert abs(g[h + 2, h + 3] / g[h, h] - math.exp(-(9 / (2 * 1.3 ** 2) + 4 / (2 * 0.7 ** 2)))) < 1e-14


def test_kernel_zero_sigma_is_delta():
    g = ora.gaussian_kernel(0.0, 0.0, 11)
    d = np.zeros((11, 11))
    d[5, 5] = 1
    np.testing.assert_array_equal(g, d)
    g1 = ora.gaussian_kernel(0.0, 1.0, 5)
    assert np.all(g1[:, [0, 1, 3, 4]] == 0)
    with pytest.raises(ValueError):
        ora.gaussian_kernel(1.0, 1.0, 10)


def test_blur_conserves_total_and_constants(rng):
    g = ora.gaussian_kernel(1.0, 2.0, 11)
    a = rng.random((24, 24))
    assert abs(ora.blur_periodic(a, g).sum() - a.sum()) < 1e-12 * a.sum()
    np.testing.assert_allclose(ora.blur_periodic(np.full((16, 16), 3.5), g), 3.5, atol=1e-14)


def test_blur_equals_separable_and_fft_convolution(rng):
    n = 20
    s1, s2 = 1.1, 1.7
    g = ora.gaussian_kernel(s1, s2, 11)
    a = rng.random((n, n))
    out = ora.blur_periodic(a, g)
    # separable two-pass, written from the 1D factors of Eq. (7)
    d = np.arange(-5, 6)
    gx = np.exp(-d ** 2 / (2 * s1 ** 2)); gx /= gx.sum()
    gy = np.exp(-d ** 2 / (2 * s2 ** 2)); gy /= gy.sum()
    tmp = np.zeros_like(a)
    for i, dx in enumerate(d):
        tmp += gx[i] * np.roll(a, dx, axis=1)
    sep = np.zeros_like(a)
    for i, dy in enumerate(d):
        sep += gy[i] * np.roll(tmp, dy, axis=0)
    np.testing.assert_allclose(out, sep, atol=1e-14)
    # convolution theorem on the periodic grid
    kern = np.zeros((n, n))
    for iy, dy in enumerate(d):
        for ix, dx in enumerate(d):
            kern[dy % n, dx % n] += g[iy, ix]
    viafft = np.real(np.fft.ifft2(np.fft.fft2(a) * np.fft.fft2(kern)))
    np.testing.assert_allclose(out, viafft, atol=1e-13)


def test_blur_impulse_response():
    n = 16
    a = np.zeros((n, n))
    a[3, 14] = 1.0
    g = ora.gaussian_kernel(0.9, 1.4, 7)
    out = ora.blur_periodic(a, g)
    for dy in range(-3, 4):
        for dx in range(-3, 4):
            assert abs(out[(3 + dy) % n, (14 + dx) % n] - g[dy + 3, dx + 3]) < 1e-15


def _psi(rng, k, n):
    return rng.standard_normal((k, n, n)) + 1j * rng.standard_normal((k, n, n))


@pytest.mark.parametrize("domain", [ora.BLUR_AMPLITUDE, ora.BLUR_INTENSITY])
def test_consistent_data_gives_zero_update(domain, rng):
    n, k = 16, 3
    p = ora.Params(n=n, n_modes=k, sigma1=1.2, sigma2=0.8, blur_domain=domain, eps=0.0)
    g = ora.gaussian_kernel(p.sigma1, p.sigma2, p.kernel_size)
    Psi = _psi(rng, k, n)
    i_mod = np.sum(np.abs(Psi) ** 2, axis=0)
    # build data by a route independent of the oracle's: FFT-circular convolution
    d = np.arange(-5, 6)
    kern = np.zeros((n, n))
    for iy, dy in enumerate(d):
        for ix, dx in enumerate(d):
            kern[dy % n, dx % n] += g[iy, ix]
    conv = lambda f: np.real(np.fft.ifft2(np.fft.fft2(f) * np.fft.fft2(kern)))
    meas = conv(np.sqrt(i_mod)) if domain == ora.BLUR_AMPLITUDE else np.sqrt(conv(i_mod))
    Psi_new, factor, ag = ora.modulus_constraint(Psi, meas, p, g)
    np.testing.assert_allclose(factor, 1.0, atol=1e-12)
    np.testing.assert_allclose(Psi_new, Psi, atol=1e-12)


def test_coherent_limit_imposes_measured_modulus(rng):
    n = 16
    p = ora.Params(n=n, sigma1=0.0, sigma2=0.0, eps=0.0)
    Psi = _psi(rng, 1, n)
    meas = rng.random((n, n)) * 3
    Psi_new, _, _ = ora.modulus_constraint(Psi, meas, p)
    np.testing.assert_allclose(np.abs(Psi_new[0]), meas, atol=1e-13)
    np.testing.assert_allclose(np.angle(Psi_new[0]), np.angle(Psi[0]), atol=1e-12)


def test_unitary_mode_mixing_invariance(rng):
    n, k = 12, 3
    p = ora.Params(n=n, n_modes=k, sigma1=1.0, sigma2=1.0)
    Psi = _psi(rng, k, n)
    q, _ = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    mixed = np.tensordot(q, Psi, axes=(1, 0))
    meas = rng.random((n, n))
    _, f1, _ = ora.modulus_constraint(Psi, meas, p)
    _, f2, _ = ora.modulus_constraint(mixed, meas, p)
    np.testing.assert_allclose(f1, f2, rtol=1e-12)
