"""ctypes binding of include/ptycho_ws.h: the learned warm start (argument
marshalling only; the network, its training, the features, the rendered probe
and the training-set generator all run in the HIP library).

Device arrays are torch CUDA tensors; every call is ordered on torch's
current stream.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np

from .ptycho import PTYCHO_MEM_DEVICE, PTYCHO_MEM_HOST, PTYCHO_OK, PtychoError, load_library

try:
    import torch
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

__all__ = [
    "PTYCHO_WS_SIDE", "PTYCHO_WS_OUTPUTS", "PTYCHO_WS_N_PARAMS", "FmConfig", "ws_library",
    "ptycho_ws_param_count", "ptycho_ws_features", "ptycho_ws_render_probe", "WarmStartNet",
    "ForwardModel", "TARGET_NAMES", "TARGET_OFFSET", "TARGET_SCALE", "WarmStart", "predict_settings",
]

PTYCHO_WS_SIDE, PTYCHO_WS_OUTPUTS, PTYCHO_WS_N_PARAMS = 128, 4, 46692
TARGET_NAMES = ("sigma", "bandwidth", "radius", "defocus")
# training targets are uniform on these ranges; the network regresses (t - off) / scale
_RANGES = ((0.5, 3.0), (0.0, 0.05), (12.0, 20.0), (0.5, 2.0))
TARGET_OFFSET = tuple(0.5 * (a + b) for a, b in _RANGES)
TARGET_SCALE = tuple((b - a) / math.sqrt(12.0) for a, b in _RANGES)


class FmConfig(ctypes.Structure):
    _fields_ = [
        ("obj_side", ctypes.c_int32), ("n_scan", ctypes.c_int32), ("step", ctypes.c_int32),
        ("jitter", ctypes.c_int32), ("n_wl", ctypes.c_int32), ("counts", ctypes.c_float),
        ("sigma_lo", ctypes.c_float), ("sigma_hi", ctypes.c_float), ("bw_lo", ctypes.c_float),
        ("bw_hi", ctypes.c_float), ("r_lo", ctypes.c_float), ("r_hi", ctypes.c_float),
        ("c_lo", ctypes.c_float), ("c_hi", ctypes.c_float),
    ]


_ws_lib = None


def ws_library():
    global _ws_lib
    if _ws_lib is not None:
        return _ws_lib
    L = load_library()
    P = ctypes.POINTER
    vp, i32, i64, u64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
    sig = {
        "ptycho_ws_param_count": (i32, []),
        "ptycho_ws_create": (i32, [i32, vp, P(vp)]),
        "ptycho_ws_set_params": (i32, [vp, vp, i32]),
        "ptycho_ws_get_params": (i32, [vp, vp, i32]),
        "ptycho_ws_set_target_scaling": (i32, [vp, P(f32), P(f32)]),
        "ptycho_ws_forward": (i32, [vp, vp, vp, i32, vp]),
        "ptycho_ws_loss_grad": (i32, [vp, vp, vp, vp, i32, P(f32), vp, i32]),
        "ptycho_ws_train_step": (i32, [vp, vp, vp, vp, i32, f32, P(f32)]),
        "ptycho_ws_reset_optimizer": (i32, [vp]),
        "ptycho_ws_destroy": (None, [vp]),
        "ptycho_ws_last_error": (ctypes.c_char_p, []),
        "ptycho_ws_features": (i32, [vp, i32, i32, vp, vp]),
        "ptycho_ws_render_probe": (i32, [i32, i32, f32, f32, f32, vp, vp]),
        "ptycho_fm_default_config": (None, [P(FmConfig)]),
        "ptycho_fm_create": (i32, [P(FmConfig), i32, vp, P(vp)]),
        "ptycho_fm_generate": (i32, [vp, u64, i64, i32, vp, vp]),
        "ptycho_fm_patterns": (i32, [vp, vp, vp, i32, f32, f32, f32, f32, vp]),
        "ptycho_fm_objects": (i32, [vp, u64, i64, i32, vp]),
        "ptycho_fm_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _ws_lib = L
    return L


def _check(status):
    if status != PTYCHO_OK:
        msg = ws_library().ptycho_ws_last_error()
        raise PtychoError(status, msg.decode() if msg else "")


def _dev(t, dtype):
    """Device pointer of a contiguous CUDA tensor of the given dtype."""
    if not (torch is not None and isinstance(t, torch.Tensor) and t.is_cuda):
        raise ValueError("expected a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def _inputs(x, target, idx, nb, max_batch):
    """Check shapes and indices of a network call; returns the batch size."""
    if x.dim() != 3 or tuple(x.shape[1:]) != (PTYCHO_WS_SIDE, PTYCHO_WS_SIDE):
        raise ValueError("inputs must be [*, 128, 128]")
    if target is not None and (target.dim() != 2 or target.shape[1] != PTYCHO_WS_OUTPUTS
                               or target.shape[0] != x.shape[0]):
        raise ValueError("targets must be [len(inputs), 4]")
    if idx is not None:
        if idx.dim() != 1 or idx.dtype != torch.int32:
            raise ValueError("idx must be a 1-D int32 tensor")
        nb = idx.numel()
        if nb and (int(idx.min()) < 0 or int(idx.max()) >= x.shape[0]):
            raise ValueError("idx out of range of the inputs")
    elif nb is None:
        nb = x.shape[0]
    elif nb > x.shape[0]:
        raise ValueError("nb exceeds the number of inputs")
    if not 1 <= nb <= max_batch:
        raise ValueError(f"batch {nb} outside [1, {max_batch}]")
    return int(nb)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def ptycho_ws_param_count():
    return int(ws_library().ptycho_ws_param_count())


def ptycho_ws_features(intensities):
    """intensities: CUDA float32 [n_pat, n, n] -> CUDA float32 [128, 128] network input."""
    if intensities.dim() != 3 or intensities.shape[1] != intensities.shape[2]:
        raise ValueError("intensities must be [n_pat, n, n]")
    n_pat, n, _ = intensities.shape
    out = torch.empty((PTYCHO_WS_SIDE, PTYCHO_WS_SIDE), dtype=torch.float32, device=intensities.device)
    _check(ws_library().ptycho_ws_features(_dev(intensities, torch.float32), n_pat, n, _dev(out, torch.float32),
                                           _stream()))
    return out


def ptycho_ws_render_probe(n, n_modes, radius, defocus, total_power, device="cuda"):
    """-> CUDA complex64 [n_modes, n, n]."""
    out = torch.empty((n_modes, n, n), dtype=torch.complex64, device=device)
    _check(ws_library().ptycho_ws_render_probe(n, n_modes, float(radius), float(defocus), float(total_power),
                                               ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


class WarmStartNet:
    """The warm-start network (ptycho_ws_*)."""

    def __init__(self, max_batch=256, params=None, normalise=True):
        L = ws_library()
        h = ctypes.c_void_p()
        _check(L.ptycho_ws_create(int(max_batch), _stream(), ctypes.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        self.y = torch.empty((self.max_batch, PTYCHO_WS_OUTPUTS), dtype=torch.float32, device="cuda")
        if normalise:
            self.set_target_scaling(TARGET_OFFSET, TARGET_SCALE)
        if params is not None:
            self.set_params(params)

    def set_target_scaling(self, off, scale):
        o = (ctypes.c_float * 4)(*[float(v) for v in off])
        s = (ctypes.c_float * 4)(*[float(v) for v in scale])
        _check(ws_library().ptycho_ws_set_target_scaling(self._h, o, s))

    def set_params(self, theta):
        if isinstance(theta, np.ndarray):
            a = np.ascontiguousarray(theta, dtype=np.float32)
            if a.size != PTYCHO_WS_N_PARAMS:
                raise ValueError("wrong parameter count")
            _check(ws_library().ptycho_ws_set_params(self._h, ctypes.c_void_p(a.ctypes.data), PTYCHO_MEM_HOST))
        else:
            if theta.numel() != PTYCHO_WS_N_PARAMS:
                raise ValueError("wrong parameter count")
            _check(ws_library().ptycho_ws_set_params(self._h, _dev(theta, torch.float32), PTYCHO_MEM_DEVICE))

    def get_params(self):
        a = np.empty(PTYCHO_WS_N_PARAMS, dtype=np.float32)
        _check(ws_library().ptycho_ws_get_params(self._h, ctypes.c_void_p(a.ctypes.data), PTYCHO_MEM_HOST))
        return a

    def forward(self, x, idx=None, nb=None):
        """x: CUDA float32 [*, 128, 128]; idx: optional CUDA int32 [nb] -> CUDA float32 [nb, 4]."""
        nb = _inputs(x, None, idx, nb, self.max_batch)
        ip = _dev(idx, torch.int32) if idx is not None else None
        _check(ws_library().ptycho_ws_forward(self._h, _dev(x, torch.float32), ip, nb, _dev(self.y, torch.float32)))
        return self.y[:nb].clone()

    def loss_grad(self, x, target, idx=None, nb=None):
        """-> (loss, gradient as a float32 numpy vector in the parameter order)."""
        nb = _inputs(x, target, idx, nb, self.max_batch)
        ip = _dev(idx, torch.int32) if idx is not None else None
        g = np.empty(PTYCHO_WS_N_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        _check(ws_library().ptycho_ws_loss_grad(self._h, _dev(x, torch.float32), ip, _dev(target, torch.float32), nb,
                                                ctypes.byref(loss), ctypes.c_void_p(g.ctypes.data), PTYCHO_MEM_HOST))
        return float(loss.value), g

    def train_step(self, x, target, idx=None, lr=1e-3, nb=None, want_loss=False):
        nb = _inputs(x, target, idx, nb, self.max_batch)
        ip = _dev(idx, torch.int32) if idx is not None else None
        loss = ctypes.c_float()
        _check(ws_library().ptycho_ws_train_step(self._h, _dev(x, torch.float32), ip, _dev(target, torch.float32), nb,
                                                 float(lr), ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def reset_optimizer(self):
        _check(ws_library().ptycho_ws_reset_optimizer(self._h))

    def close(self):
        if getattr(self, "_h", None):
            ws_library().ptycho_ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class ForwardModel:
    """GPU generator of (network input, target) training pairs (ptycho_fm_*)."""

    def __init__(self, max_chunk=512, **overrides):
        L = ws_library()
        cfg = FmConfig()
        L.ptycho_fm_default_config(ctypes.byref(cfg))
        for k, v in overrides.items():
            if not hasattr(cfg, k):
                raise AttributeError(k)
            setattr(cfg, k, v)
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(L.ptycho_fm_create(ctypes.byref(cfg), int(max_chunk), _stream(), ctypes.byref(h)))
        self._h = h
        self.max_chunk = int(max_chunk)

    def generate(self, seed, first, count, feat=None, targets=None):
        """Samples [first, first + count) -> (feat CUDA [count,128,128], targets CUDA [count,4]); views of the
        given output tensors when passed."""
        if not 1 <= count <= self.max_chunk:
            raise ValueError(f"count {count} outside [1, {self.max_chunk}]")
        if feat is None:
            feat = torch.empty((count, PTYCHO_WS_SIDE, PTYCHO_WS_SIDE), dtype=torch.float32, device="cuda")
        if targets is None:
            targets = torch.empty((count, PTYCHO_WS_OUTPUTS), dtype=torch.float32, device="cuda")
        if tuple(feat.shape) != (count, PTYCHO_WS_SIDE, PTYCHO_WS_SIDE) or tuple(targets.shape) != (count, 4):
            raise ValueError("output tensors must be [count, 128, 128] and [count, 4]")
        _check(ws_library().ptycho_fm_generate(self._h, int(seed) & (2 ** 64 - 1), int(first), int(count),
                                               _dev(feat, torch.float32), _dev(targets, torch.float32)))
        return feat, targets

    def objects(self, seed, first, count):
        side = self.cfg.obj_side
        out = torch.empty((count, side, side, 2), dtype=torch.float32, device="cuda")
        _check(ws_library().ptycho_fm_objects(self._h, int(seed) & (2 ** 64 - 1), int(first), int(count),
                                              _dev(out, torch.float32)))
        return out

    def patterns(self, log_amp_phase, positions, sigma, bandwidth, radius, defocus):
        """Noise-free patterns of one object: log_amp_phase CUDA float32 [side, side, 2], positions host
        int32 [n_pos, 2] -> CUDA float32 [n_pos, 64, 64]."""
        pos = np.ascontiguousarray(positions, dtype=np.int32)
        side = self.cfg.obj_side
        if tuple(log_amp_phase.shape) != (side, side, 2):
            raise ValueError(f"object must be [{side}, {side}, 2]")
        if pos.ndim != 2 or pos.shape[1] != 2:
            raise ValueError("positions must be [n_pos, 2]")
        out = torch.empty((len(pos), 64, 64), dtype=torch.float32, device="cuda")
        _check(ws_library().ptycho_fm_patterns(self._h, _dev(log_amp_phase, torch.float32),
                                               ctypes.c_void_p(pos.ctypes.data), len(pos), float(sigma),
                                               float(bandwidth), float(radius), float(defocus),
                                               _dev(out, torch.float32)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            ws_library().ptycho_fm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class WarmStart:
    """Settings predicted for one scan: blur sigma, bandwidth, aperture radius, defocus,
    the mode count they imply and the rendered initial probe."""

    def __init__(self, sigma, bandwidth, radius, defocus, n_modes, probe):
        self.sigma, self.bandwidth, self.radius, self.defocus = sigma, bandwidth, radius, defocus
        self.n_modes = n_modes
        self.probe = probe

    def as_dict(self):
        return dict(sigma=self.sigma, bandwidth=self.bandwidth, radius=self.radius, defocus=self.defocus,
                    n_modes=self.n_modes)


def predict_settings(net, intensities, multi_mode_bandwidth=0.01, max_modes=4):
    """Warm start for one far-field scan (intensities CUDA float32 [n_pat, n, n], zero frequency
    at the centre): features -> network -> (sigma, bandwidth, radius, defocus), clamped to the
    trained ranges; K = max_modes if the predicted bandwidth exceeds multi_mode_bandwidth else 1;
    the probe is rendered with the mean pattern total as its power."""
    n = intensities.shape[-1]
    x = ptycho_ws_features(intensities)
    y = net.forward(x.unsqueeze(0), nb=1)[0].cpu().numpy().astype(np.float64)
    vals = [min(max(float(v), lo), hi) for v, (lo, hi) in zip(y, _RANGES)]
    sigma, bw, radius, defocus = vals
    k = max_modes if bw > multi_mode_bandwidth else 1
    total = float(intensities.sum(dim=(1, 2)).mean().item())
    probe = ptycho_ws_render_probe(n, k, radius * n / 64.0, defocus, total)
    return WarmStart(sigma, bw, radius * n / 64.0, defocus, k, probe)
