"""FP64 reference of the warm start's data side (test infrastructure only).

* the broadband far-field pattern of one scan position: for each wavelength
  scale s = lambda_c / lambda the object exp(s (ln A + i phi)) (the object's
  log-amplitude and phase scale inversely with wavelength, Eq. 15-16) times the
  probe, transformed by the centred DFT whose frequencies are scaled by s (the
  pattern of a longer wavelength is magnified, Sec. 3.1), the intensities
  summed with equal weights over the wavelengths, then convolved with the
  normalised periodic Gaussian of Eq. 2 and 7 on the full frame;
* the network input: the mean over a scan's patterns of log(1 + I), centred
  (zero frequency at the middle), standardised over the frame and zero-padded
  to a larger square;
* the rendered warm-start probe: an aperture of radius R with a quadratic phase
  2 pi c r^2 / N^2, plus extra incoherent modes made from it by the odd
  multipliers x, y and x y (orthogonal to it and to each other by symmetry).

Written as plain dense sums so that each can be read against its definition.
"""

from __future__ import annotations

import math

import numpy as np

N_WAVELENGTHS = 5
EXTRA_MODE_POWER = 0.05


def wavelength_scales(bandwidth, n_wl=N_WAVELENGTHS):
    """Scales s_j = 1 / (1 + d_j), d_j evenly spaced over [-bandwidth/2, bandwidth/2]."""
    if n_wl == 1:
        return np.array([1.0])
    d = np.linspace(-bandwidth / 2.0, bandwidth / 2.0, n_wl)
    return 1.0 / (1.0 + d)


def scaled_dft_matrix(n, s):
    """F[u, x] = exp(-2 pi i s (u - n/2)(x - n/2) / n) / sqrt(n)."""
    c = np.arange(n) - n / 2.0
    return np.exp(-2j * math.pi * s * np.outer(c, c) / n) / math.sqrt(n)


def scaled_dft2(x, s):
    """Centred 2D DFT with frequency scale s: F x F^T (unitary at s = 1)."""
    f = scaled_dft_matrix(x.shape[-1], s)
    return f @ x @ f.T


def periodic_gaussian_1d(n, sigma):
    """Normalised periodic Gaussian g[d] ~ exp(-min(d, n-d)^2 / (2 sigma^2)), full support."""
    d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
    g = np.exp(-d * d / (2.0 * sigma * sigma))
    return g / g.sum()


def blur_periodic_full(img, sigma):
    """Circular convolution of img with the separable normalised Gaussian (Eq. 2, 7)."""
    n = img.shape[-1]
    g = periodic_gaussian_1d(n, sigma)
    out = np.zeros_like(img, dtype=np.float64)
    tmp = np.zeros_like(img, dtype=np.float64)
    for d in range(n):
        tmp += g[d] * np.roll(img, d, axis=-1)
    for d in range(n):
        out += g[d] * np.roll(tmp, d, axis=-2)
    return out


def farfield_pattern(log_amp, phase, probe, scales, sigma):
    """Noise-free pattern of one position: sum_j |F_s (exp(s_j (lnA + i phi)) P)|^2 / J, blurred."""
    acc = np.zeros(probe.shape, dtype=np.float64)
    for s in scales:
        o = np.exp(s * (log_amp + 1j * phase))
        psi = scaled_dft2(o * probe, s)
        acc += np.abs(psi) ** 2
    acc /= len(scales)
    return blur_periodic_full(acc, sigma) if sigma > 0 else acc


def aperture(n, radius, defocus):
    """Disc of radius R about (n/2, n/2) times exp(i 2 pi c r^2 / n^2)."""
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    r2 = (x - n / 2.0) ** 2 + (y - n / 2.0) ** 2
    return np.where(r2 <= radius * radius, np.exp(2j * math.pi * defocus * r2 / (n * n)), 0.0)


def render_probe(n, n_modes, radius, defocus, total_power):
    """K modes: base x {1, x^, y^, x^ y^} (x^ = (x - n/2)/(n/4)), each normalised, with
    powers proportional to (1, 0.05, 0.05, 0.05) and summing to total_power."""
    base = aperture(n, radius, defocus)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    xh = (x - n / 2.0) / (n / 4.0)
    yh = (y - n / 2.0) / (n / 4.0)
    mult = [np.ones_like(xh), xh, yh, xh * yh]
    pw = np.array([1.0] + [EXTRA_MODE_POWER] * (n_modes - 1))
    pw = pw / pw.sum() * total_power
    modes = []
    for k in range(n_modes):
        m = base * mult[k]
        nrm = math.sqrt(float(np.sum(np.abs(m) ** 2)))
        modes.append(m / nrm * math.sqrt(pw[k]) if nrm > 0 else m)
    return np.stack(modes)


def features(intensities, out_side):
    """Network input: mean_n log(1 + I_n) (frames already centred), standardised
    over the frame (mean 0, standard deviation 1; a frame whose standard
    deviation is at most 1e-6 (1 + |mean|), i.e. constant up to rounding, maps to 0),
    placed in the middle of an out_side x out_side zero image."""
    n = intensities.shape[-1]
    m = np.mean(np.log1p(np.asarray(intensities, dtype=np.float64)), axis=0)
    mu = m.mean()
    sd = m.std()
    z = (m - mu) / sd if sd > 1e-6 * (1.0 + abs(mu)) else np.zeros_like(m)
    out = np.zeros((out_side, out_side))
    o = (out_side - n) // 2
    out[o:o + n, o:o + n] = z
    return out
