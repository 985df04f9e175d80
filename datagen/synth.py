"""Synthetic scans shaped like the paper's workloads (seeded, numpy).

Recipes (all readings where the paper is silent; each is listed in the design
notes):

* object: amplitude and phase each drawn as N(0, 1) noise, low-passed with a
  periodic Gaussian of sigma = 3 px, then min-max mapped to [0.8, 1] and
  [-pi/2, pi/2] respectively;
* probe: a circular aperture times a quadratic defocus phase 2 pi r^2 / D^2
  (D the frame side), optionally times a low-passed random phase screen
  (structured illumination, Sec. 4.3); extra incoherent modes are the base mode
  times low-order polynomials, orthonormalised and given the requested powers;
* scan: raster with integer jitter, centred in the object;
* far-field data: |DFT(o P_k)|^2 summed over modes and wavelengths (the
  object's ln A and phase scale with lambda_c / lambda, Eq. 15-16; the pattern
  scales with wavelength, Sec. 3.1), convolved with a normalised full-support
  periodic Gaussian (Eq. 2), scaled to a mean total count, Poisson noise, zero
  frequency at (N/2, N/2);
* near-field data: paraxial free-space propagation with pixel Fresnel number
  F_px, same blur and noise.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

__all__ = [
    "object_texture", "aperture_probe", "probe_modes", "raster_positions",
    "farfield_intensities", "nearfield_intensities", "initial_guess",
    "make_scan", "CONFIGS", "random_case_spec",
]

_WORKERS = -1


def _lowpass(noise, sigma):
    """Periodic Gaussian low-pass of a real field (generation only)."""
    h, w = noise.shape
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    tf = np.exp(-2.0 * (math.pi * sigma) ** 2 * (fx ** 2 + fy ** 2))
    return np.real(sfft.ifft2(sfft.fft2(noise, workers=_WORKERS) * tf, workers=_WORKERS))


def _minmax(x, lo, hi):
    x = (x - x.min()) / max(x.max() - x.min(), 1e-300)
    return lo + (hi - lo) * x


def object_texture(shape, rng, amp=(0.8, 1.0), phase=(-math.pi / 2, math.pi / 2), sigma=3.0):
    a = _minmax(_lowpass(rng.standard_normal(shape), sigma), *amp)
    p = _minmax(_lowpass(rng.standard_normal(shape), sigma), *phase)
    return a * np.exp(1j * p)


def aperture_probe(n, radius, defocus=1.0, rng=None, screen_sigma=None):
    """Circular aperture of `radius` px centred at (n/2, n/2) times exp(i 2 pi defocus r^2 / n^2);
    with `rng` and `screen_sigma`, also times a uniform random phase screen low-passed
    by a Gaussian of screen_sigma px (a tissue-covered pinhole, Sec. 4.3)."""
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    r2 = (x - n / 2) ** 2 + (y - n / 2) ** 2
    p = (r2 <= radius * radius).astype(np.complex128)
    p *= np.exp(1j * 2 * math.pi * defocus * r2 / (n * n))
    if rng is not None and screen_sigma is not None:
        screen = _lowpass(rng.uniform(-math.pi, math.pi, (n, n)), screen_sigma)
        screen = _minmax(screen, -math.pi, math.pi)
        p *= np.exp(1j * screen)
    return p


_POLY = [
    lambda x, y: np.ones_like(x), lambda x, y: x, lambda x, y: y, lambda x, y: x * y,
    lambda x, y: x * x, lambda x, y: y * y, lambda x, y: x * x * y, lambda x, y: x * y * y,
]


def probe_modes(base, k, powers, total_power=1.0):
    """K mutually orthogonal modes: base x {1, x, y, xy, x^2, y^2, x^2 y, x y^2},
    orthonormalised (QR) and scaled so that mode k carries powers[k] * total_power."""
    n = base.shape[0]
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    x = (x - n / 2) / (n / 4)
    y = (y - n / 2) / (n / 4)
    cols = np.stack([(base * _POLY[i](x, y)).ravel() for i in range(k)], axis=1)
    q, _ = np.linalg.qr(cols)
    modes = np.ascontiguousarray(q.T).reshape(k, n, n)
    # fix the sign of each mode so it overlaps positively with its generator
    for i in range(k):
        ov = np.vdot(modes[i], base * _POLY[i](x, y))
        if abs(ov) > 0:
            modes[i] *= ov / abs(ov)
    pw = np.asarray(powers, dtype=np.float64)
    pw = pw / pw.sum()
    return modes * np.sqrt(pw * total_power)[:, None, None]


def raster_positions(n_side, step, jitter, n, obj_shape, rng):
    """n_side x n_side raster of top-left (row, col) corners, integer jitter in
    [-jitter, jitter], centred in the object and clipped to stay inside it."""
    extent = (n_side - 1) * step + n
    r0 = (obj_shape[0] - extent) // 2
    c0 = (obj_shape[1] - extent) // 2
    pos = []
    for i in range(n_side):
        for j in range(n_side):
            dr, dc = (rng.integers(-jitter, jitter + 1, 2) if jitter > 0 else (0, 0))
            r = min(max(r0 + i * step + int(dr), 0), obj_shape[0] - n)
            c = min(max(c0 + j * step + int(dc), 0), obj_shape[1] - n)
            pos.append((r, c))
    return np.array(pos, dtype=np.int32)


def _periodic_gaussian_tf(n, sigma):
    if sigma <= 0:
        return None
    d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
    g1 = np.exp(-d * d / (2 * sigma * sigma))
    g = g1[:, None] * g1[None, :]
    g /= g.sum()
    return sfft.fft2(g, workers=_WORKERS)


def _blur_counts(i_stack, sigma, counts, rng):
    tf = _periodic_gaussian_tf(i_stack.shape[-1], sigma)
    if tf is not None:
        i_stack = np.real(sfft.ifft2(sfft.fft2(i_stack, axes=(-2, -1), workers=_WORKERS) * tf,
                                     axes=(-2, -1), workers=_WORKERS))
    i_stack = np.maximum(i_stack, 0.0)
    scale = counts / max(np.mean(np.sum(i_stack, axis=(-2, -1))), 1e-300)
    i_stack = i_stack * scale
    if rng is not None:
        i_stack = rng.poisson(i_stack).astype(np.float64)
    return i_stack.astype(np.float32)


class _ScaledDFT2:
    """Centred 2D DFT with frequency scale s, unitary at s = 1:
    X(v~, u~) = N^-1 sum_{y~,x~} x(y~, x~) exp(-2 pi i s (u~ x~ + v~ y~) / N),
    u~ = u - N/2, x~ = x - N/2.  Evaluated by the chirp-z identity
    u x = (u^2 + x^2 - (u - x)^2) / 2 as a linear convolution through 2N x 2N FFTs."""

    def __init__(self, n, s):
        c = np.arange(n) - n / 2
        ch = np.exp(-1j * math.pi * s * c * c / n)
        self.chirp = (ch[:, None] * ch[None, :]).astype(np.complex64)
        d = np.concatenate([np.arange(n), np.arange(-n, 0)]).astype(np.float64)
        kf = sfft.fft(np.exp(1j * math.pi * s * d * d / n))
        self.kf = (kf[:, None] * kf[None, :] / n).astype(np.complex64)
        self.n = n

    def __call__(self, x):
        n = self.n
        a = x * self.chirp
        y = sfft.fft2(a, s=(2 * n, 2 * n), axes=(-2, -1), workers=1)
        y *= self.kf
        y = sfft.ifft2(y, axes=(-2, -1), workers=1, overwrite_x=True)[..., :n, :n]
        return y * self.chirp


def farfield_intensities(obj, modes, positions, sigma, counts, rng, wavelength_scales=(1.0,),
                         weights=None, chunk=8):
    """Far-field recorded intensities, zero frequency at (N/2, N/2).

    For wavelength scale s = lambda_c / lambda the exit wave uses the object
    exp(s (ln A + i phi)) and is transformed by the centred DFT with
    frequencies scaled by s (the pattern-scaling of a broadband source)."""
    k, n, _ = modes.shape
    n_pos = len(positions)
    if weights is None:
        weights = np.full(len(wavelength_scales), 1.0 / len(wavelength_scales))
    log_obj = np.log(np.where(np.abs(obj) > 0, obj, 1e-300))
    objs = {s: np.exp(s * log_obj).astype(np.complex64) for s in wavelength_scales}
    out = np.zeros((n_pos, n, n), dtype=np.float64)
    m64 = modes.astype(np.complex64)
    dfts = {s: _ScaledDFT2(n, s) for s in wavelength_scales if s != 1.0}

    def work(s0):
        sl = positions[s0:s0 + chunk]
        acc = np.zeros((len(sl), n, n), dtype=np.float64)
        for s, wgt in zip(wavelength_scales, weights):
            o = np.stack([objs[s][r:r + n, c:c + n] for (r, c) in sl])
            psi = o[:, None] * m64[None]
            if s == 1.0:
                Psi = sfft.fftshift(sfft.fft2(psi, axes=(-2, -1), norm="ortho", workers=1),
                                    axes=(-2, -1))
            else:
                Psi = dfts[s](psi)
            acc += wgt * np.sum(Psi.real ** 2 + Psi.imag ** 2, axis=1, dtype=np.float64)
        out[s0:s0 + len(sl)] = acc

    _parallel(work, range(0, n_pos, chunk))
    # blur in FFT order and centred order agree for a periodic kernel
    return _blur_counts(out, sigma, counts, rng)


def _parallel(fn, items):
    import concurrent.futures as cf
    import os
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(fn, items))


def nearfield_intensities(obj, modes, positions, fresnel_px, sigma, counts, rng, chunk=16):
    """Near-field recorded intensities: paraxial free-space propagation with
    transfer function exp(-i pi (u^2 + v^2) / (N^2 F_px)) (signed indices)."""
    k, n, _ = modes.shape
    f = np.fft.fftfreq(n, d=1.0 / n)
    h1 = np.exp(-1j * math.pi * f * f / (n * n * fresnel_px))
    tf = (h1[:, None] * h1[None, :]).astype(np.complex64)
    out = np.zeros((len(positions), n, n), dtype=np.float64)
    m64 = modes.astype(np.complex64)
    for s0 in range(0, len(positions), chunk):
        sl = positions[s0:s0 + chunk]
        o = np.stack([obj[r:r + n, c:c + n] for (r, c) in sl]).astype(np.complex64)
        psi = o[:, None] * m64[None]
        Psi = sfft.ifft2(sfft.fft2(psi, axes=(-2, -1), workers=_WORKERS) * tf, axes=(-2, -1),
                         workers=_WORKERS)
        out[s0:s0 + len(sl)] = np.sum(np.abs(Psi.astype(np.complex128)) ** 2, axis=1)
    return _blur_counts(out, sigma, counts, rng)


def initial_guess(obj_shape, n, k, radius, intensities, defocus=0.0):
    """Plain-method start: O = 1; P_0 = the aperture with flat phase (or the given
    defocus), power-matched to the mean pattern total; extra modes are the base
    times polynomials at 5 % of the power each."""
    base = aperture_probe(n, radius, defocus=defocus)
    total = float(np.mean(np.sum(np.asarray(intensities, dtype=np.float64), axis=(-2, -1))))
    if k == 1:
        p = base[None] * math.sqrt(total / np.sum(np.abs(base) ** 2))
    else:
        powers = [1.0] + [0.05] * (k - 1)
        p = probe_modes(base, k, powers, total_power=total)
    return np.ones(obj_shape, dtype=np.complex128), p


# ----------------------------------------------------------------------------
# The workload configurations
# ----------------------------------------------------------------------------

CONFIGS = {
    # far field, 64^2 frames, 10x10 raster at 8 px; object enlarged to 144^2 so the
    # scan extent 9*8 + 64 + 2 fits
    "far64": dict(seed=1001, geometry=0, obj=(144, 144), n=64, n_side=10, step=8, jitter=1, k=1, powers=(1.0,),
               radius=16, defocus=1.0, sigma_data=1.0, counts=1e5, wavelengths=(1.0,),
               sigma=1.0, batch=1, iterations=50, screen=None, fresnel_px=0.0),
    # far field, 256^2 frames, 40x40 raster at 16 px, 4 modes, 5 wavelengths +-2.5 %
    "far256_k4": dict(seed=1002, geometry=0, obj=(1024, 1024), n=256, n_side=40, step=16, jitter=1, k=4,
               powers=(0.6, 0.25, 0.1, 0.05), radius=64, defocus=1.0, sigma_data=2.0, counts=1e6,
               wavelengths=tuple(1.0 / (1.0 + s) for s in (-0.025, -0.0125, 0.0, 0.0125, 0.025)),
               sigma=2.0, batch=32, iterations=200, screen=None, fresnel_px=0.0),
    # near field, 512^2 frames, 15x15 raster at 60 +- 10 px, 8 modes, F_px = 20 / 70^2
    "near512_k8": dict(seed=1003, geometry=1, obj=(1536, 1536), n=512, n_side=15, step=60, jitter=10, k=8,
               powers=tuple(2.0 ** -i for i in range(8)), radius=70, defocus=0.0, sigma_data=1.5,
               counts=1e6, wavelengths=(1.0,), sigma=1.5, batch=8, iterations=100, screen=2.0,
               fresnel_px=20.0 / 70.0 ** 2),
}


def random_case_spec(i):
    """Case i of the 64-case batched workload: N in {64,128,192,256}, 100-2500
    positions, 1-8 modes (seeded by [1004, i])."""
    rng = np.random.default_rng(np.random.SeedSequence([1004, i]))
    n = int(rng.choice([64, 128, 192, 256]))
    n_pos = int(rng.integers(100, 2501))
    k = int(rng.integers(1, 9))
    n_side = int(math.ceil(math.sqrt(n_pos)))
    step = n // 8
    extent = (n_side - 1) * step + n + 2
    side = int(math.ceil(extent / 16.0) * 16)
    return dict(geometry=0, obj=(side, side), n=n, n_side=n_side, step=step, jitter=1, k=k,
                powers=tuple(2.0 ** -j for j in range(k)), radius=n // 4, defocus=1.0,
                sigma_data=1.0, counts=1e5, wavelengths=(1.0,), sigma=1.0, batch=32,
                iterations=100, screen=None, fresnel_px=0.0, n_pos=n_pos, seed_key=[1004, i])


def make_scan(spec, seed, noise=True, n_pos=None, probe_known=False):
    """Build one synthetic scan from a config dict.

    Returns a dict with: obj_true [H,W] c128, probe_true [K,N,N] c128,
    positions [n_pos,2] int32, intensities [n_pos,N,N] f32 (zero frequency
    centred for far field), obj0, probe0 (plain initial guess), and the
    reconstruction settings (n, k, geometry, fresnel_px, sigma, batch).
    """
    ss = np.random.SeedSequence(seed)
    r_amp, r_probe, r_jit, r_noise, r_misc = [np.random.default_rng(s) for s in ss.spawn(5)]
    n, k = spec["n"], spec["k"]
    obj = object_texture(spec["obj"], r_amp)
    base = aperture_probe(n, spec["radius"], spec["defocus"], rng=r_probe if spec.get("screen") else None,
                          screen_sigma=spec.get("screen"))
    # power scale so that sum |P|^2 ~ 1 per pixel of the aperture (counts set later)
    if k == 1:
        modes = base[None] / math.sqrt(np.sum(np.abs(base) ** 2))
    else:
        modes = probe_modes(base, k, spec["powers"])
    pos = raster_positions(spec["n_side"], spec["step"], spec["jitter"], n, spec["obj"], r_jit)
    want = spec.get("n_pos", n_pos)
    if n_pos is not None:
        want = n_pos
    if want is not None:
        pos = pos[:want]
    rng_noise = r_noise if noise else None
    if spec["geometry"] == 0:
        ints = farfield_intensities(obj, modes, pos, spec["sigma_data"], spec["counts"], rng_noise,
                                    wavelength_scales=spec["wavelengths"])
    else:
        ints = nearfield_intensities(obj, modes, pos, spec["fresnel_px"], spec["sigma_data"],
                                     spec["counts"], rng_noise)
    total = float(np.mean(np.sum(ints.astype(np.float64), axis=(-2, -1))))
    # rescale the true probe to the measured power (unitary propagators conserve it)
    modes = modes * math.sqrt(total / max(np.sum(np.abs(modes) ** 2), 1e-300))
    o0, p0 = initial_guess(spec["obj"], n, k, spec["radius"], ints)
    if probe_known:
        p0 = modes.copy()
    return dict(obj_true=obj, probe_true=modes, positions=pos, intensities=ints, obj0=o0,
                probe0=p0, n=n, k=k, geometry=spec["geometry"], fresnel_px=spec["fresnel_px"],
                sigma=spec["sigma"], batch=spec["batch"], iterations=spec["iterations"])
