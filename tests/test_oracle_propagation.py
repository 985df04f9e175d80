"""Pins for the oracle's propagators (Eq. 1; near-field geometry of Sec. 3.1).

Each check is fixed by mathematics independent of the oracle's code: a
brute-force DFT, Parseval, the shift theorem, and the closed-form width of a
paraxial Gaussian beam.
"""

import math

import numpy as np
import pytest

import oracle as ora


def _brute_dft2(x):
    n = x.shape[-1]
    out = np.zeros_like(x, dtype=np.complex128)
    for v in range(n):
        for u in range(n):
            acc = 0j
            for y in range(n):
                for xx in range(n):
                    acc += x[y, xx] * complex(math.cos(-2 * math.pi * (u * xx + v * y) / n),
                                              math.sin(-2 * math.pi * (u * xx + v * y) / n))
            out[v, u] = acc / n
    return out


@pytest.mark.parametrize("n", [8, 12])
def test_fft_equals_brute_force_dft(n, rng):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    np.testing.assert_allclose(ora.fft2u(x), _brute_dft2(x), atol=1e-12)


def test_parseval_and_inverse(rng):
    x = rng.standard_normal((3, 32, 32)) + 1j * rng.standard_normal((3, 32, 32))
    X = ora.fft2u(x)
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2)) < 1e-12 * np.sum(np.abs(x) ** 2)
    np.testing.assert_allclose(ora.ifft2u(X), x, atol=1e-13)


def test_impulse_and_shift_theorem(rng):
    n = 16
    d = np.zeros((n, n), complex)
    d[0, 0] = 1
    np.testing.assert_allclose(ora.fft2u(d), np.full((n, n), 1.0 / n), atol=1e-15)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    sy, sx = 3, 5
    xs = np.roll(x, (sy, sx), axis=(0, 1))
    u = np.arange(n)
    ramp = np.exp(-2j * math.pi * (u[None, :] * sx + u[:, None] * sy) / n)
    np.testing.assert_allclose(ora.fft2u(xs), ora.fft2u(x) * ramp, atol=1e-12)


def _near(n, f):
    return ora.Params(n=n, geometry=ora.NEAR_FIELD, fresnel_px=f)


def test_nearfield_unitary_and_inverse(rng):
    n = 32
    p = _near(n, 0.01)
    h = ora.transfer_function(n, 0.01)
    np.testing.assert_allclose(np.abs(h), 1.0, atol=1e-14)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = ora.propagate(x, p)
    assert abs(np.linalg.norm(y) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    np.testing.assert_allclose(ora.backpropagate(y, p), x, atol=1e-12)


def test_nearfield_large_fresnel_is_identity(rng):
    n = 32
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    np.testing.assert_allclose(ora.propagate(x, _near(n, 1e12)), x, atol=1e-9)


def test_nearfield_distances_add(rng):
    # 1/F_px is proportional to z, so z1 followed by z2 equals z1 + z2
    n = 32
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    f1, f2 = 0.02, 0.05
    f12 = 1.0 / (1.0 / f1 + 1.0 / f2)
    two = ora.propagate(ora.propagate(x, _near(n, f1)), _near(n, f2))
    np.testing.assert_allclose(two, ora.propagate(x, _near(n, f12)), atol=1e-11)


def test_nearfield_gaussian_beam_width():
    """Paraxial Gaussian beam: u0 = exp(-r^2 / w0^2) spreads to
    w(z)^2 = w0^2 (1 + (z / z_R)^2) with z / z_R = 1 / (pi w0^2 F_px) in pixel units,
    so the intensity second moment per axis is w(z)^2 / 4."""
    n = 256
    w0 = 6.0
    f_px = 1.0 / (math.pi * w0 * w0 * 1.5)  # z = 1.5 z_R
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r2 = (x - n / 2) ** 2 + (y - n / 2) ** 2
    u0 = np.exp(-r2 / (w0 * w0)).astype(complex)
    u = ora.propagate(u0, _near(n, f_px))
    inten = np.abs(u) ** 2
    mx = np.sum(inten * (x - n / 2) ** 2) / np.sum(inten)
    wz2 = w0 * w0 * (1 + 1.5 ** 2)
    assert abs(mx - wz2 / 4) < 1e-6 * wz2
    # wrong constants (2 pi instead of pi, or N instead of N^2) change the width grossly
    assert abs(mx - w0 * w0 / 4) > 0.5 * w0 * w0


def test_farfield_propagation_roundtrip(rng):
    p = ora.Params(n=16)
    x = rng.standard_normal((2, 16, 16)) + 1j * rng.standard_normal((2, 16, 16))
    np.testing.assert_allclose(ora.backpropagate(ora.propagate(x, p), p), x, atol=1e-13)
