"""Evaluation of reconstructions of synthetic scans whose true object is known:
the object error NMSE, wall time and iterations to an NMSE threshold, for the
plain start and for the learned warm start, run singly or as one batched group.

NMSE = min_c sum_ROI |c O_rec - O_true|^2 / sum_ROI |O_true|^2 with the global
complex scalar c = <O_rec, O_true> / ||O_rec||^2 removed; the ROI is the set of
pixels whose summed true illumination sum_n sum_k |P_k(r - r_n)|^2 is at least a
tenth of its maximum.  Ptychography leaves a linear phase ramp between object
and probe undetermined (O e^{ig.r}, P e^{-ig.r} explain the same data), so a
second error, nmse_ramp, also removes the best ramp g.  The clock runs from the start of initialisation with the
data in host memory (for the warm start it includes the features, the
network and the probe rendering) to the end of each iteration; the NMSE itself
is evaluated outside it, after every iteration.
"""

from __future__ import annotations

import math
import os
import time

import numpy as np

from . import learned as L
from .ptycho import PTYCHO_MEM_DEVICE, Group, Reconstruction, default_params

try:
    import torch
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warm_start.npz")


def illumination_roi(positions, probe, obj_shape, frac=0.1):
    n = probe.shape[-1]
    illum = np.zeros(obj_shape)
    p2 = np.sum(np.abs(probe) ** 2, axis=0)
    for r, c in positions:
        illum[int(r):int(r) + n, int(c):int(c) + n] += p2
    return illum >= frac * illum.max()


def nmse(o_rec, o_true, roi):
    a = np.asarray(o_rec, dtype=np.complex128)[roi]
    b = np.asarray(o_true, dtype=np.complex128)[roi]
    den = np.vdot(a, a).real
    c = np.vdot(a, b) / den if den > 0 else 0.0
    return float(np.sum(np.abs(c * a - b) ** 2) / np.sum(np.abs(b) ** 2))


def nmse_ramp(o_rec, o_true, roi):
    """min over a global complex scalar c and a linear phase ramp g of
    sum_ROI |c e^{i g.r} O_rec - O_true|^2 / sum_ROI |O_true|^2.  The ramp starts at
    the peak of the cross-spectrum of O_true conj(O_rec) on a 4x zero-padded grid and
    is refined by Nelder-Mead; c is closed-form for each ramp."""
    import scipy.optimize
    a = np.asarray(o_rec, dtype=np.complex128)[roi]
    b = np.asarray(o_true, dtype=np.complex128)[roi]
    yy, xx = np.nonzero(roi)
    bb = float(np.sum(np.abs(b) ** 2))
    if not np.any(a) or bb == 0:
        return nmse(o_rec, o_true, roi)

    def err(g):
        ar = a * np.exp(1j * (g[0] * yy + g[1] * xx))
        c = np.vdot(ar, b) / np.vdot(ar, ar)
        return float(np.sum(np.abs(c * ar - b) ** 2) / bb)

    h, w = roi.shape
    d = np.zeros((4 * h, 4 * w), dtype=np.complex128)
    d[yy, xx] = b * np.conj(a)
    spec = np.abs(np.fft.fft2(d))
    ky, kx = np.unravel_index(int(np.argmax(spec)), spec.shape)
    ky = ky - 4 * h if ky >= 2 * h else ky
    kx = kx - 4 * w if kx >= 2 * w else kx
    g0 = [2 * math.pi * ky / (4 * h), 2 * math.pi * kx / (4 * w)]
    res = scipy.optimize.minimize(err, g0, method="Nelder-Mead", options=dict(xatol=1e-8, fatol=1e-14))
    return min(float(res.fun), err([0.0, 0.0]))


def load_warm_start(path=DEFAULT_WEIGHTS, max_batch=1):
    """The trained network and its training report."""
    import json
    with np.load(path, allow_pickle=False) as z:
        theta = z["theta"]
        report = json.loads(str(z["report"]))
    return L.WarmStartNet(max_batch=max_batch, params=theta), report


def _params(scan, sigma, n_modes, batch, seed, blur_domain=0):
    h, w = scan["obj0"].shape
    p = default_params(n=scan["n"], n_modes=n_modes, n_pos=len(scan["positions"]), obj_h=h, obj_w=w,
                       sigma1=float(sigma), sigma2=float(sigma), batch=batch, seed=seed, blur_domain=blur_domain)
    p.cc_start, p.cc_end = 1, 0  # the complex constraint stays off (the objects are not homogeneous)
    return p


def _sync():
    torch.cuda.synchronize()


def start_plain(scan, sigma=1.0, batch=1, seed=1, blur_domain=0):
    """Plain start: O = 1, the scan's plain probe guess, blur sigma 1."""
    p = _params(scan, sigma, scan["probe0"].shape[0], batch, seed, blur_domain)
    return Reconstruction(p, scan["intensities"], scan["positions"], scan["probe0"].astype(np.complex64),
                          scan["obj0"].astype(np.complex64)), None


def start_learned(net, scan, batch=1, seed=1, multi_mode_bandwidth=0.01, blur_domain=0):
    """Warm start: patterns to the GPU, features, network, rendered probe, then init from device memory."""
    ints = torch.from_numpy(np.ascontiguousarray(scan["intensities"], dtype=np.float32)).cuda()
    ws = L.predict_settings(net, ints, multi_mode_bandwidth=multi_mode_bandwidth)
    p = _params(scan, ws.sigma, ws.n_modes, batch, seed, blur_domain)
    pos = torch.from_numpy(np.ascontiguousarray(scan["positions"], dtype=np.int32)).cuda()
    obj = torch.ones(scan["obj0"].shape, dtype=torch.complex64, device="cuda")
    rec = Reconstruction(p, ints, pos, ws.probe, obj, mem_kind=PTYCHO_MEM_DEVICE)
    return rec, ws


def trace_single(make, scan, n_iter, err=nmse):
    """[(iteration, wall_s, error)] for one reconstruction started by make(); error = err(...)."""
    roi = illumination_roi(scan["positions"], scan["probe_true"], scan["obj_true"].shape)
    _sync()
    t0 = time.perf_counter()
    rec, info = make()
    _sync()
    wall = time.perf_counter() - t0
    out = [(0, wall, err(rec.object(), scan["obj_true"], roi))]
    try:
        for it in range(1, n_iter + 1):
            t1 = time.perf_counter()
            rec.iterate(1)
            wall += time.perf_counter() - t1
            out.append((it, wall, err(rec.object(), scan["obj_true"], roi)))
    finally:
        rec.close()
    return out, info


def trace_group(makers, scans, n_iter, graph=True, err=nmse):
    """One batched group of reconstructions advanced together (iterations replayed from a
    captured graph when `graph`); per case [(iteration, wall_s, nmse)] on the group's shared clock."""
    rois = [illumination_roi(s["positions"], s["probe_true"], s["obj_true"].shape) for s in scans]
    _sync()
    t0 = time.perf_counter()
    started = [m() for m in makers]
    recs = [r for r, _ in started]
    grp = Group(recs)
    grp.set_graph(graph)
    _sync()
    wall = time.perf_counter() - t0
    traces = [[(0, wall, err(r.object(), s["obj_true"], roi))] for r, s, roi in zip(recs, scans, rois)]
    try:
        for it in range(1, n_iter + 1):
            t1 = time.perf_counter()
            grp.iterate(1)
            wall += time.perf_counter() - t1
            for tr, r, s, roi in zip(traces, recs, scans, rois):
                tr.append((it, wall, err(r.object(), s["obj_true"], roi)))
    finally:
        grp.close()
        for r in recs:
            r.close()
    return traces, [i for _, i in started]


def time_to(trace, tau):
    """(iterations, wall_s) of the first point of trace with NMSE <= tau, or None."""
    for it, wall, e in trace:
        if e <= tau:
            return it, wall
    return None


def compare(plain, learned):
    """Smallest NMSE both traces reach and the iterations / wall time each needs for it."""
    tau = max(min(e for _, _, e in plain), min(e for _, _, e in learned))
    tp, tl = time_to(plain, tau), time_to(learned, tau)
    return dict(threshold=tau, plain_iterations=tp[0], plain_wall_s=tp[1], learned_iterations=tl[0],
                learned_wall_s=tl[1], plain_final_nmse=plain[-1][2], learned_final_nmse=learned[-1][2])


def log10_or_none(v):
    return None if v is None or v <= 0 else math.log10(v)


SIGMA_SWEEP = (0.5, 1.0, 2.0, 3.0)


def sweep_report(net, scans, sigmas, n_iter):
    """Plain vs learned (single, eager) per case, and learned + batched (one group, graph
    replay) over the sweep: the smallest NMSE both single variants reach per case, the
    iterations and wall time each needs, and the wall time the group needs until every case
    has reached its threshold against the plain runs one after another."""
    s0 = scans[0]
    trace_single(lambda: start_plain(s0), s0, 1)  # first-call costs out of the clock
    trace_single(lambda: start_learned(net, s0), s0, 1)
    cases, plain_total = [], 0.0
    for sd, s in zip(sigmas, scans):
        tp, _ = trace_single(lambda: start_plain(s), s, n_iter)
        tl, ws = trace_single(lambda: start_learned(net, s), s, n_iter)
        c = compare(tp, tl)
        c.update(sigma_data=sd, predicted={k: round(v, 4) if isinstance(v, float) else v
                                           for k, v in ws.as_dict().items()})
        cases.append(c)
        plain_total += c["plain_wall_s"]
    trace_group([lambda s=s: start_learned(net, s) for s in scans[:1]], scans[:1], 1)
    tg, _ = trace_group([lambda s=s: start_learned(net, s) for s in scans], scans, n_iter)
    group_wall = 0.0
    for c, tr in zip(cases, tg):
        hit = time_to(tr, c["threshold"])
        c["learned_batched_iterations"] = hit[0] if hit else None
        group_wall = max(group_wall, hit[1] if hit else float("inf"))
    return dict(cases=cases, plain_sequential_wall_s=plain_total, learned_batched_wall_s=group_wall,
                speedup=plain_total / group_wall if group_wall > 0 else None, iterations=n_iter)


def threshold_report(net, scans, sigmas, n_iter, tau=1e-3, blur_domain=1, err=nmse_ramp):
    """Wall seconds (and iterations) to the object error `tau` itself: plain start (blur
    sigma 1) per case one after another, against the learned start of every case advanced
    as one group with graph replay.  A case that does not reach tau within n_iter
    iterations reports None; the totals cover the cases both variants reach."""
    s0 = scans[0]
    trace_single(lambda: start_plain(s0, blur_domain=blur_domain), s0, 1, err)
    trace_group([lambda s=s: start_learned(net, s, blur_domain=blur_domain) for s in scans[:1]], scans[:1], 1,
                err=err)
    cases = []
    for sd, s in zip(sigmas, scans):
        tp, _ = trace_single(lambda: start_plain(s, blur_domain=blur_domain), s, n_iter, err)
        hp = time_to(tp, tau)
        cases.append(dict(sigma_data=sd, plain_iterations=hp[0] if hp else None, plain_wall_s=hp[1] if hp else None,
                          plain_final=tp[-1][2]))
    tg, infos = trace_group([lambda s=s: start_learned(net, s, blur_domain=blur_domain) for s in scans], scans,
                            n_iter, err=err)
    for c, tr, ws in zip(cases, tg, infos):
        hl = time_to(tr, tau)
        c.update(learned_batched_iterations=hl[0] if hl else None, learned_batched_wall_s=hl[1] if hl else None,
                 learned_final=tr[-1][2], predicted={k: round(v, 4) if isinstance(v, float) else v
                                                     for k, v in ws.as_dict().items()})
    both = [c for c in cases if c["plain_wall_s"] is not None and c["learned_batched_wall_s"] is not None]
    plain_total = sum(c["plain_wall_s"] for c in both)
    group_wall = max((c["learned_batched_wall_s"] for c in both), default=0.0)
    return dict(threshold=tau, cases=cases, cases_both_reach=len(both),
                cases_plain_reaches=sum(c["plain_wall_s"] is not None for c in cases),
                cases_learned_reaches=sum(c["learned_batched_wall_s"] is not None for c in cases),
                plain_sequential_wall_s=plain_total, learned_batched_wall_s=group_wall,
                speedup=plain_total / group_wall if both and group_wall > 0 else None, iterations=n_iter)
