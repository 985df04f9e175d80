"""Seeded far-field scans generated with torch on a GPU (input synthesis only).

The same recipe as `synth.make_scan` for single-wavelength far-field configs:
object, probe, modes and raster come from the numpy generators of `synth`;
the patterns |FFT(o P_k)|^2 summed over modes, the normalised periodic
Gaussian blur (Eq. 2, full frame), the count scaling and the Poisson draw run
as torch operations on the device, so that many large scans (the 64-case
batched workload) are generated in seconds.  The Poisson draws come from a
torch generator seeded from the scan seed, so a scan is reproducible on one
device type; it is not bitwise the numpy scan of the same seed.
"""

from __future__ import annotations

import math

import numpy as np

from . import synth


def _blur_tf(n, sigma, device):
    import torch
    d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
    g1 = np.exp(-d * d / (2 * sigma * sigma))
    g = g1[:, None] * g1[None, :]
    g /= g.sum()
    return torch.fft.fft2(torch.from_numpy(g).to(device=device, dtype=torch.complex64))


def farfield_intensities(obj, modes, positions, sigma, counts, seed, device="cuda", chunk=64):
    """Far-field patterns [n_pos][N][N] float32 on `device`, zero frequency at (N/2, N/2)."""
    import torch
    k, n, _ = modes.shape
    o = torch.from_numpy(np.asarray(obj, dtype=np.complex64)).to(device)
    m = torch.from_numpy(np.asarray(modes, dtype=np.complex64)).to(device)
    pos = np.asarray(positions)
    out = torch.empty((len(pos), n, n), dtype=torch.float32, device=device)
    tf = _blur_tf(n, sigma, device) if sigma > 0 else None
    rows = torch.arange(n, device=device)
    for s0 in range(0, len(pos), chunk):
        sl = torch.from_numpy(pos[s0:s0 + chunk].astype(np.int64)).to(device)
        r = (sl[:, 0, None] + rows[None, :])[:, :, None]
        c = (sl[:, 1, None] + rows[None, :])[:, None, :]
        boxes = o[r, c]
        psi = boxes[:, None] * m[None]
        inten = torch.fft.fft2(psi, norm="ortho").abs().square().sum(dim=1)
        if tf is not None:
            inten = torch.fft.ifft2(torch.fft.fft2(inten.to(torch.complex64)) * tf).real
        out[s0:s0 + len(sl)] = torch.fft.fftshift(inten.clamp_min(0.0), dim=(-2, -1))
    scale = counts / max(float(out.sum(dim=(-2, -1)).mean().item()), 1e-30)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(np.random.SeedSequence(seed).generate_state(1)[0]))
    return torch.poisson(out * scale, generator=gen)


def make_scan(spec, seed, device="cuda"):
    """`synth.make_scan` for a single-wavelength far-field spec with the patterns made on the GPU
    (returned as a device tensor under "intensities_dev"; "intensities" is the host copy)."""
    if spec["geometry"] != 0 or tuple(spec["wavelengths"]) != (1.0,):
        raise ValueError("the GPU generator covers single-wavelength far-field scans")
    ss = np.random.SeedSequence(seed)
    r_amp, r_probe, r_jit, r_noise, r_misc = [np.random.default_rng(s) for s in ss.spawn(5)]
    n, k = spec["n"], spec["k"]
    obj = synth.object_texture(spec["obj"], r_amp)
    base = synth.aperture_probe(n, spec["radius"], spec["defocus"])
    modes = base[None] / math.sqrt(np.sum(np.abs(base) ** 2)) if k == 1 else synth.probe_modes(base, k, spec["powers"])
    pos = synth.raster_positions(spec["n_side"], spec["step"], spec["jitter"], n, spec["obj"], r_jit)
    if spec.get("n_pos") is not None:
        pos = pos[:spec["n_pos"]]
    ints = farfield_intensities(obj, modes, pos, spec["sigma_data"], spec["counts"], seed, device)
    total = float(ints.sum(dim=(-2, -1)).mean().item())
    modes = modes * math.sqrt(total / max(np.sum(np.abs(modes) ** 2), 1e-300))
    ints_host = ints.cpu().numpy()
    o0, p0 = synth.initial_guess(spec["obj"], n, k, spec["radius"], ints_host)
    return dict(obj_true=obj, probe_true=modes, positions=pos, intensities=ints_host, intensities_dev=ints,
                obj0=o0, probe0=p0, n=n, k=k, geometry=0, fresnel_px=0.0, sigma=spec["sigma"],
                batch=spec["batch"], iterations=spec["iterations"])
