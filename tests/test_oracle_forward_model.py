"""Pins for the warm start's data-side reference (oracle/forward_model.py):
the scaled DFT against numpy's FFT at s = 1 and against the chirp-z evaluation
used by the input generator at s != 1, the blur against an FFT convolution,
Parseval, the feature standardisation and the orthogonality of rendered modes."""

import math

import numpy as np
import scipy.fft as sfft

import datagen
from datagen import synth
from oracle import forward_model as fm


def test_scaled_dft_unit_scale_is_shifted_fft(rng):
    n = 16
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    got = fm.scaled_dft2(x, 1.0)
    ref = np.fft.fftshift(np.fft.fft2(x, norm="ortho"))
    sign = (-1.0) ** (np.arange(n) - n // 2)
    np.testing.assert_allclose(got, sign[:, None] * sign[None, :] * ref, atol=1e-12)
    assert abs(np.sum(np.abs(got) ** 2) - np.sum(np.abs(x) ** 2)) < 1e-9


def test_scaled_dft_matches_chirp_z(rng):
    n = 32
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    for s in (0.975, 1.0128):
        got = fm.scaled_dft2(x, s)
        ref = synth._ScaledDFT2(n, s)(x.astype(np.complex64)[None])[0]
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


def test_wavelength_scales_match_broadband_config():
    got = fm.wavelength_scales(0.05)
    np.testing.assert_allclose(got, datagen.CONFIGS["far256_k4"]["wavelengths"], rtol=1e-14)
    np.testing.assert_allclose(fm.wavelength_scales(0.0), np.ones(5))


def test_blur_matches_fft_convolution(rng):
    n = 24
    img = rng.random((n, n))
    for sigma in (0.5, 1.7, 3.0):
        got = fm.blur_periodic_full(img, sigma)
        d = np.minimum(np.arange(n), n - np.arange(n)).astype(float)
        g = np.exp(-d[:, None] ** 2 / (2 * sigma ** 2) - d[None, :] ** 2 / (2 * sigma ** 2))
        g /= g.sum()
        ref = np.real(sfft.ifft2(sfft.fft2(img) * sfft.fft2(g)))
        np.testing.assert_allclose(got, ref, atol=1e-12)
        assert abs(got.sum() - img.sum()) < 1e-10


def test_pattern_parseval_and_blur_total(rng):
    n = 16
    la = 0.1 * rng.standard_normal((n, n))
    ph = rng.standard_normal((n, n))
    p = fm.aperture(n, 5, 1.0)
    i0 = fm.farfield_pattern(la, ph, p, [1.0], 0.0)
    assert abs(i0.sum() - np.sum(np.abs(np.exp(la + 1j * ph) * p) ** 2)) < 1e-9
    i1 = fm.farfield_pattern(la, ph, p, [1.0], 1.5)
    assert abs(i1.sum() - i0.sum()) < 1e-9
    # all scales equal to one reduce to the single-wavelength pattern
    np.testing.assert_allclose(fm.farfield_pattern(la, ph, p, [1.0] * 5, 1.5), i1, atol=1e-12)


def test_features_standardised_and_padded(rng):
    ints = rng.poisson(50.0, (7, 16, 16)).astype(np.float32)
    f = fm.features(ints, 32)
    c = f[8:24, 8:24]
    assert abs(c.mean()) < 1e-12 and abs(c.std() - 1.0) < 1e-12
    assert np.all(f[:8] == 0) and np.all(f[24:] == 0) and np.all(f[:, :8] == 0)
    ref = np.log1p(ints.astype(float)).mean(0)
    np.testing.assert_allclose(c, (ref - ref.mean()) / ref.std(), atol=1e-12)
    assert np.all(fm.features(np.full((3, 16, 16), 4.0), 32) == 0)


def test_rendered_modes_orthogonal_with_powers():
    n = 64
    for radius, c in ((12.0, 0.5), (20.0, 2.0), (16.0, 1.0)):
        p = fm.render_probe(n, 4, radius, c, 1000.0)
        g = np.einsum("kyx,lyx->kl", p.conj(), p)
        pw = np.array([1, 0.05, 0.05, 0.05]) / 1.15 * 1000.0
        np.testing.assert_allclose(np.diag(g).real, pw, rtol=1e-12)
        off = g - np.diag(np.diag(g))
        assert np.max(np.abs(off)) < 1e-9 * 1000.0
        # the first mode is the disc with the stated quadratic phase
        y, x = np.mgrid[0:n, 0:n]
        r2 = (x - n / 2) ** 2 + (y - n / 2) ** 2
        inside = r2 <= radius ** 2
        ph = np.angle(p[0][inside] * np.exp(-2j * math.pi * c * r2[inside] / n ** 2))
        assert np.max(np.abs(ph)) < 1e-12
        assert np.all(p[0][~inside] == 0)
