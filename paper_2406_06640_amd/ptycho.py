"""ctypes binding of the C ABI in include/ptycho.h (argument marshalling only).

Functions keep the C names.  Array arguments may be numpy arrays (host memory)
or torch CUDA tensors (device memory); complex arrays are complex64, which has
the interleaved (re, im) float layout the library expects.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # torch must load the HIP runtime before the library does (one runtime per process)
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

__all__ = [
    "PTYCHO_OK", "PTYCHO_E_INVALID", "PTYCHO_E_SHAPE", "PTYCHO_E_OOM", "PTYCHO_E_HIP",
    "PTYCHO_E_NUMERIC", "PTYCHO_E_STATE", "PTYCHO_FAR_FIELD", "PTYCHO_NEAR_FIELD",
    "PTYCHO_BLUR_AMPLITUDE", "PTYCHO_BLUR_INTENSITY", "PTYCHO_MEM_HOST", "PTYCHO_MEM_DEVICE",
    "PTYCHO_ENGINE_EPIE", "PTYCHO_ENGINE_DM", "PTYCHO_ENGINE_LSQML", "ptycho_get_exit_waves", "ptycho_set_exit_waves",
    "ptycho_get_lsq_steps",
    "ptycho_mono_create", "ptycho_mono_run", "ptycho_mono_destroy", "Monochromatiser",
    "PtychoParams", "PtychoError", "lib", "library_path", "load_library", "default_params",
    "ptycho_init", "ptycho_iterate", "ptycho_iterate_static", "ptycho_get_object", "ptycho_get_probe", "ptycho_set_state",
    "ptycho_iteration", "ptycho_debug_step", "ptycho_destroy", "ptycho_last_error",
    "ptycho_permutation", "ptycho_set_timing", "ptycho_kernel_time", "kernel_names",
    "ptycho_set_graph", "ptycho_set_variant", "ptycho_variant_count", "ptycho_autotune", "ptycho_dft2_bf16", "ptycho_group_create", "ptycho_group_iterate",
    "ptycho_group_destroy", "ptycho_group_last_error", "ptycho_group_set_graph", "Reconstruction", "Group",
]

PTYCHO_OK, PTYCHO_E_INVALID, PTYCHO_E_SHAPE, PTYCHO_E_OOM = 0, -1, -2, -3
PTYCHO_E_HIP, PTYCHO_E_NUMERIC, PTYCHO_E_STATE = -4, -5, -6
PTYCHO_FAR_FIELD, PTYCHO_NEAR_FIELD = 0, 1
PTYCHO_BLUR_AMPLITUDE, PTYCHO_BLUR_INTENSITY = 0, 1
PTYCHO_ENGINE_EPIE, PTYCHO_ENGINE_DM, PTYCHO_ENGINE_LSQML = 0, 1, 2
PTYCHO_MEM_HOST, PTYCHO_MEM_DEVICE = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.environ.get("PTYCHO_LIB", os.path.join(_HERE, "_lib", "libptycho.so"))


class PtychoParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_modes", ctypes.c_int32), ("n_pos", ctypes.c_int32),
        ("obj_h", ctypes.c_int32), ("obj_w", ctypes.c_int32),
        ("geometry", ctypes.c_int32), ("fresnel_px", ctypes.c_double),
        ("sigma1", ctypes.c_float), ("sigma2", ctypes.c_float), ("kernel_size", ctypes.c_int32),
        ("blur_domain", ctypes.c_int32), ("eps", ctypes.c_float),
        ("alpha1", ctypes.c_float), ("alpha2", ctypes.c_float),
        ("cbar_min", ctypes.c_float), ("cbar_max", ctypes.c_float),
        ("cc_start", ctypes.c_int32), ("cc_end", ctypes.c_int32), ("cc_period", ctypes.c_int32),
        ("obj_step", ctypes.c_float), ("probe_step", ctypes.c_float),
        ("gamma_obj", ctypes.c_float), ("gamma_probe", ctypes.c_float),
        ("probe_update_start", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("orthogonalize", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("dft_bf16", ctypes.c_int32),
        ("engine", ctypes.c_int32), ("dm_reg", ctypes.c_float), ("lsq_damping", ctypes.c_float),
    ]


class PtychoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"ptycho status {status}: {message}")
        self.status = status


_lib = None


def load_library():
    """Load libptycho.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or paper_2406_06640_amd/build.py)")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i32, u32, u64, fp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    sig = {
        "ptycho_default_params": (None, [P(PtychoParams)]),
        "ptycho_init": (i32, [P(PtychoParams), fp, fp, fp, fp, i32, vp, P(vp)]),
        "ptycho_iterate": (i32, [vp, i32, fp, fp]),
        "ptycho_iterate_static": (i32, [vp, i32, fp, fp]),
        "ptycho_get_exit_waves": (i32, [vp, fp, i32]),
        "ptycho_get_lsq_steps": (i32, [vp, fp, fp]),
        "ptycho_mono_create": (i32, [i32, i32, fp, fp, i32, vp, P(vp)]),
        "ptycho_mono_run": (i32, [vp, fp, fp, i32, i32, fp, i32]),
        "ptycho_mono_destroy": (None, [vp]),
        "ptycho_set_exit_waves": (i32, [vp, fp, i32]),
        "ptycho_get_object": (i32, [vp, fp, i32]),
        "ptycho_get_probe": (i32, [vp, fp, i32]),
        "ptycho_set_state": (i32, [vp, fp, fp, i32, i32]),
        "ptycho_iteration": (i32, [vp]),
        "ptycho_debug_step": (i32, [vp, fp, i32, i32, fp, fp, fp, fp, fp, fp, fp, i32]),
        "ptycho_set_timing": (i32, [vp, u32]),
        "ptycho_kernel_time": (i32, [vp, i32, P(ctypes.c_double), P(ctypes.c_int64), i32]),
        "ptycho_kernel_name": (ctypes.c_char_p, [i32]),
        "ptycho_kernel_class_count": (i32, []),
        "ptycho_destroy": (None, [vp]),
        "ptycho_last_error": (ctypes.c_char_p, [vp]),
        "ptycho_permutation": (i32, [u64, i32, i32, fp]),
        "ptycho_set_graph": (i32, [vp, i32]),
        "ptycho_set_variant": (i32, [vp, i32]),
        "ptycho_variant_count": (i32, []),
        "ptycho_dft2_bf16": (i32, [fp, i32, i32, i32, vp]),
        "ptycho_autotune": (i32, [vp, i32, i32, P(i32)]),
        "ptycho_group_create": (i32, [P(vp), i32, P(vp)]),
        "ptycho_group_iterate": (i32, [vp, i32, fp]),
        "ptycho_group_set_graph": (i32, [vp, i32]),
        "ptycho_group_destroy": (None, [vp]),
        "ptycho_group_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def lib():
    return load_library()


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _is_torch(x):
    return torch is not None and isinstance(x, torch.Tensor)


def _ptr(x, dtype, mem_kind, keep):
    """Pointer to x's data; numpy arrays are made contiguous with `dtype`."""
    if x is None:
        return None
    if _is_torch(x):
        if mem_kind != PTYCHO_MEM_DEVICE or not x.is_cuda:
            raise ValueError("torch tensors must be CUDA tensors passed with PTYCHO_MEM_DEVICE")
        x = x.contiguous()
        keep.append(x)
        return ctypes.c_void_p(x.data_ptr())
    if mem_kind != PTYCHO_MEM_HOST:
        raise ValueError("numpy arrays are host memory: use PTYCHO_MEM_HOST")
    a = np.ascontiguousarray(x, dtype=dtype)
    keep.append(a)
    return ctypes.c_void_p(a.ctypes.data)


def _check(status, ctx=None):
    if status != PTYCHO_OK:
        msg = load_library().ptycho_last_error(ctx)
        raise PtychoError(status, msg.decode() if msg else "")


def default_params(**kw) -> PtychoParams:
    p = PtychoParams()
    load_library().ptycho_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _stream_handle(stream):
    if stream is None:
        return None
    if _is_torch_stream(stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _is_torch_stream(s):
    return torch is not None and isinstance(s, torch.cuda.Stream)


# ---------------------------------------------------------------------------
# C entry points (same names)
# ---------------------------------------------------------------------------

def ptycho_init(params, intensities, positions, probe0, object0, mem_kind=PTYCHO_MEM_HOST, stream=None):
    L = load_library()
    keep = []
    out = ctypes.c_void_p()
    st = L.ptycho_init(ctypes.byref(params), _ptr(intensities, np.float32, mem_kind, keep),
                       _ptr(positions, np.int32, mem_kind, keep), _ptr(probe0, np.complex64, mem_kind, keep),
                       _ptr(object0, np.complex64, mem_kind, keep), mem_kind, _stream_handle(stream),
                       ctypes.byref(out))
    _check(st, None)
    return out


def ptycho_iterate(ctx, n_iter, order=None):
    L = load_library()
    keep = []
    err = np.zeros(max(int(n_iter), 1), dtype=np.float32)
    st = L.ptycho_iterate(ctx, int(n_iter), _ptr(order, np.int32, PTYCHO_MEM_HOST, keep),
                          ctypes.c_void_p(err.ctypes.data))
    _check(st, ctx)
    return err[:n_iter]


def ptycho_iterate_static(ctx, n_iter, order=None):
    """ptycho_iterate with every per-call buffer in the library's static scratch (no allocation)."""
    L = load_library()
    keep = []
    err = np.zeros(max(int(n_iter), 1), dtype=np.float32)
    st = L.ptycho_iterate_static(ctx, int(n_iter), _ptr(order, np.int32, PTYCHO_MEM_HOST, keep),
                                 ctypes.c_void_p(err.ctypes.data))
    _check(st, ctx)
    return err[:n_iter]


def ptycho_get_object(ctx, out):
    mk = PTYCHO_MEM_DEVICE if _is_torch(out) else PTYCHO_MEM_HOST
    _check(load_library().ptycho_get_object(ctx, _out_ptr(out, mk), mk), ctx)
    return out


def ptycho_get_probe(ctx, out):
    mk = PTYCHO_MEM_DEVICE if _is_torch(out) else PTYCHO_MEM_HOST
    _check(load_library().ptycho_get_probe(ctx, _out_ptr(out, mk), mk), ctx)
    return out


def ptycho_get_exit_waves(ctx, out):
    """pc-DM exit waves [n_pos][K][n][n] complex64 into `out` (numpy or CUDA tensor)."""
    mk = PTYCHO_MEM_DEVICE if _is_torch(out) else PTYCHO_MEM_HOST
    _check(load_library().ptycho_get_exit_waves(ctx, _out_ptr(out, mk), mk), ctx)
    return out


def ptycho_get_lsq_steps(ctx, batch):
    """pc-LSQML step lengths of the last batch run: ([batch][2] (a_j, b_j), [2] means)."""
    steps = np.zeros((batch, 2), dtype=np.float32)
    mean = np.zeros(2, dtype=np.float32)
    _check(load_library().ptycho_get_lsq_steps(ctx, steps.ctypes.data, mean.ctypes.data), ctx)
    return steps, mean


def ptycho_set_exit_waves(ctx, psi, mem_kind=PTYCHO_MEM_HOST):
    keep = []
    _check(load_library().ptycho_set_exit_waves(ctx, _ptr(psi, np.complex64, mem_kind, keep), mem_kind), ctx)


def _out_ptr(x, mk):
    if x is None:
        return None
    if _is_torch(x):
        if not (x.is_cuda and x.is_contiguous()):
            raise ValueError("output tensors must be contiguous CUDA tensors")
        return ctypes.c_void_p(x.data_ptr())
    if not (isinstance(x, np.ndarray) and x.flags["C_CONTIGUOUS"] and x.flags["WRITEABLE"]):
        raise ValueError("output arrays must be writeable C-contiguous numpy arrays")
    return ctypes.c_void_p(x.ctypes.data)


def ptycho_set_state(ctx, obj=None, probe=None, iteration=0, mem_kind=PTYCHO_MEM_HOST):
    keep = []
    st = load_library().ptycho_set_state(ctx, _ptr(obj, np.complex64, mem_kind, keep),
                                         _ptr(probe, np.complex64, mem_kind, keep), int(iteration), mem_kind)
    _check(st, ctx)


def ptycho_iteration(ctx):
    return load_library().ptycho_iteration(ctx)


def ptycho_debug_step(ctx, idx, t, psi=None, psi_new=None, factor=None, n_obj=None, w_obj=None,
                      n_probe=None, v_probe=None):
    """Run one batch update over positions idx as iteration t, capturing into the given
    host arrays (complex64 / float32, shapes as in include/ptycho.h)."""
    keep = []
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    st = load_library().ptycho_debug_step(
        ctx, ctypes.c_void_p(idx.ctypes.data), len(idx), int(t),
        *[_out_ptr(a, PTYCHO_MEM_HOST) for a in (psi, psi_new, factor, n_obj, w_obj, n_probe, v_probe)],
        PTYCHO_MEM_HOST)
    del keep
    _check(st, ctx)


def ptycho_destroy(ctx):
    if ctx:
        load_library().ptycho_destroy(ctx)


def ptycho_last_error(ctx=None):
    m = load_library().ptycho_last_error(ctx)
    return m.decode() if m else ""


def ptycho_permutation(seed, t, n_pos):
    out = np.zeros(max(n_pos, 1), dtype=np.int32)
    st = load_library().ptycho_permutation(ctypes.c_uint64(seed), int(t), int(n_pos),
                                           ctypes.c_void_p(out.ctypes.data))
    _check(st, None)
    return out[:n_pos]


def ptycho_set_timing(ctx, mask):
    _check(load_library().ptycho_set_timing(ctx, int(mask)), ctx)


def ptycho_kernel_time(ctx, cls, reset=False):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load_library().ptycho_kernel_time(ctx, int(cls), ctypes.byref(ms), ctypes.byref(cnt), int(reset)), ctx)
    return ms.value, cnt.value


def kernel_names():
    L = load_library()
    return [L.ptycho_kernel_name(i).decode() for i in range(L.ptycho_kernel_class_count())]


def ptycho_dft2_bf16(frames, inverse=False, stream=None):
    """In-place unitary 2D DFT of a contiguous complex64 CUDA tensor [F][n][n] on the BF16 matrix-core path."""
    if not _is_torch(frames) or not frames.is_cuda or not frames.is_contiguous():
        raise ValueError("frames must be a contiguous complex64 CUDA tensor")
    f, n, n2 = frames.shape
    if n != n2:
        raise ValueError("frames must be square")
    _check(load_library().ptycho_dft2_bf16(ctypes.c_void_p(frames.data_ptr()), n, f, 1 if inverse else 0,
                                           _stream_handle(stream)), None)
    return frames


def ptycho_variant_count():
    return int(load_library().ptycho_variant_count())


def ptycho_set_variant(ctx, variant):
    _check(load_library().ptycho_set_variant(ctx, int(variant)), ctx)


def ptycho_set_graph(ctx, enable):
    _check(load_library().ptycho_set_graph(ctx, 1 if enable else 0), ctx)


def ptycho_autotune(ctx, trials=3, force=False):
    """Time the column-tile variants on the context's first batch; returns the chosen index."""
    chosen = ctypes.c_int32(-1)
    _check(load_library().ptycho_autotune(ctx, int(trials), 1 if force else 0, ctypes.byref(chosen)), ctx)
    return chosen.value


def ptycho_group_last_error(group=None):
    m = load_library().ptycho_group_last_error(group)
    return m.decode() if m else ""


def _gcheck(status, group):
    if status != PTYCHO_OK:
        raise PtychoError(status, ptycho_group_last_error(group))


def ptycho_group_create(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    out = ctypes.c_void_p()
    _gcheck(load_library().ptycho_group_create(arr, len(ctxs), ctypes.byref(out)), None)
    return out


def ptycho_group_iterate(group, n_iter, n_cases):
    err = np.zeros((n_cases, max(int(n_iter), 1)), dtype=np.float32)
    _gcheck(load_library().ptycho_group_iterate(group, int(n_iter), ctypes.c_void_p(err.ctypes.data)), group)
    return err[:, :n_iter] if n_iter else err[:, :0]


def ptycho_group_set_graph(group, enable):
    _gcheck(load_library().ptycho_group_set_graph(group, 1 if enable else 0), group)


def ptycho_group_destroy(group):
    if group:
        load_library().ptycho_group_destroy(group)


class Group:
    """A group of Reconstruction objects iterated together (they must outlive it)."""

    def __init__(self, recs):
        self.recs = list(recs)
        self.g = ptycho_group_create([r.ctx for r in self.recs])

    def iterate(self, n_iter):
        return ptycho_group_iterate(self.g, n_iter, len(self.recs))

    def set_graph(self, enable=True):
        ptycho_group_set_graph(self.g, enable)

    def close(self):
        if self.g:
            ptycho_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Reconstruction:
    """Owning wrapper of one context (host numpy inputs)."""

    def __init__(self, params, intensities, positions, probe0, object0, mem_kind=PTYCHO_MEM_HOST,
                 stream=None):
        self.params = params
        self.ctx = ptycho_init(params, intensities, positions, probe0, object0, mem_kind, stream)

    def iterate(self, n_iter, order=None):
        return ptycho_iterate(self.ctx, n_iter, order)

    def object(self):
        out = np.zeros((self.params.obj_h, self.params.obj_w), dtype=np.complex64)
        return ptycho_get_object(self.ctx, out)

    def probe(self):
        n = self.params.n
        out = np.zeros((self.params.n_modes, n, n), dtype=np.complex64)
        return ptycho_get_probe(self.ctx, out)

    def set_state(self, obj=None, probe=None, iteration=0):
        ptycho_set_state(self.ctx, obj, probe, iteration)

    def exit_waves(self):
        n = self.params.n
        out = np.zeros((self.params.n_pos, self.params.n_modes, n, n), dtype=np.complex64)
        return ptycho_get_exit_waves(self.ctx, out)

    def set_exit_waves(self, psi):
        ptycho_set_exit_waves(self.ctx, psi)

    def lsq_steps(self):
        """pc-LSQML: the last batch's per-position steps [batch][2] and their means [2]."""
        return ptycho_get_lsq_steps(self.ctx, self.params.batch)

    def set_graph(self, enable=True):
        ptycho_set_graph(self.ctx, enable)

    def set_variant(self, variant):
        ptycho_set_variant(self.ctx, variant)

    def autotune(self, trials=3, force=False):
        return ptycho_autotune(self.ctx, trials, force)

    @property
    def iteration(self):
        return ptycho_iteration(self.ctx)

    def close(self):
        if self.ctx:
            ptycho_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------------------
# Numerical monochromatisation by CGLS (Sec. 4.2)
# ---------------------------------------------------------------------------

def ptycho_mono_create(n, max_patterns, scales, weights, stream=None):
    sc = np.ascontiguousarray(scales, dtype=np.float32)
    wt = np.ascontiguousarray(weights, dtype=np.float32)
    if sc.shape != wt.shape or sc.ndim != 1:
        raise ValueError("scales and weights must be 1D arrays of one length")
    out = ctypes.c_void_p()
    st = load_library().ptycho_mono_create(int(n), int(max_patterns), ctypes.c_void_p(sc.ctypes.data),
                                           ctypes.c_void_p(wt.ctypes.data), int(sc.size), _stream_handle(stream),
                                           ctypes.byref(out))
    _check(st, None)
    return out


def ptycho_mono_run(handle, broadband, out, k_iters, residuals=True):
    """broadband / out: numpy float32 [P][n][n] (host) or CUDA tensors (device).  Returns the
    residual history [P][k_iters + 1] (numpy) or None."""
    mk = PTYCHO_MEM_DEVICE if _is_torch(broadband) else PTYCHO_MEM_HOST
    keep = []
    n_pat = int(broadband.shape[0])
    res = np.zeros((n_pat, int(k_iters) + 1), dtype=np.float32) if residuals else None
    st = load_library().ptycho_mono_run(handle, _ptr(broadband, np.float32, mk, keep), _out_ptr(out, mk), n_pat,
                                        int(k_iters), ctypes.c_void_p(res.ctypes.data) if residuals else None, mk)
    _check(st, None)
    return res


def ptycho_mono_destroy(handle):
    load_library().ptycho_mono_destroy(handle)


class Monochromatiser:
    """Owning wrapper of a monochromatisation plan (ptycho_mono_*)."""

    def __init__(self, n, max_patterns, scales, weights, stream=None):
        self.handle = ptycho_mono_create(n, max_patterns, scales, weights, stream)

    def run(self, broadband, out, k_iters, residuals=True):
        return ptycho_mono_run(self.handle, broadband, out, k_iters, residuals)

    def close(self):
        if getattr(self, "handle", None):
            ptycho_mono_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
