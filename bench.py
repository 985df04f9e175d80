#!/usr/bin/env python3
"""Throughput benchmark of the pc-ePIE hot path on one MI355X.

Workload: the far-field 1024^2-object scan with 256^2 frames, a 40 x 40 raster
at 16 px (1600 positions), K = 4 incoherent probe modes, 5-wavelength +-2.5 %
polychromatic data blurred by sigma = 2 px with Poisson noise at 1e6 counts
(synthetic, seeded).  One step = one full pc-ePIE iteration over all 1600
positions in batches of 32: every pass of the method runs (exit waves,
propagation, mode sum, Gaussian blur, modulus constraint, back-propagation,
object/probe updates, the complex constraint, mode orthogonalisation, the
data error).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  The metric is mode-pattern updates per second =
positions x modes x steps / wall-seconds.  Besides this headline workload the
default run also times the near-field 1536^2 / 512^2 / K = 8 workload (the
largest single-GPU configuration), the 64-case batched workload as one group,
the wall seconds to an object error of 1e-3 (plain vs learned warm start +
batching), and the FP64 oracle on the host cores.  Every leg reports its
dominant kernel against the HBM roofline and the whole iteration against the
pass-model roofline t_roof = max(B_pass / BW, F / P_FP32).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
PMC_PROFILE = os.path.join(ROOT, "profiles", "far256_k4_b32_pmc_traffic.txt")
KERNEL_SOURCES = ["kernels.hip", "kernels.hpp", "kernels_dev.hpp", "fft_lds.hpp", "dft_mfma.hip"]


def measured_traffic(kernel_class):
    """HBM bytes per launch of `kernel_class` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (scaled by its copy calibration), or None when the kernel sources changed since it was taken."""
    try:
        text = open(PMC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256: ([0-9a-f]{64})", text)
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_06640_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if not m or m.group(1) != h.hexdigest():
        return None
    m = re.search(rf"^class {re.escape(kernel_class)} traffic_bytes (\d+)$", text, re.M)
    return int(m.group(1)) if m else None


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate in GB/s (bytes read + bytes written per second) of a plain
    `nbytes` tensor copy, timed with HIP events: the achievable HBM rate the kernels can be
    compared with beside the nominal peak."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def paired_rows(n, batch):
    """Whether the pc-ePIE batch passes run the paired inverse row pass (two slots per
    workgroup, their probe contributions added on chip): power-of-two frames up to
    512 and batches of at least 2, as the library selects it."""
    return n & (n - 1) == 0 and n <= 512 and batch >= 2


def per_slot_bytes(name, n, k, near=False, pairs=False):
    """HBM bytes one batch slot (one scan position) costs in kernel `name` as the kernels are
    built, counting each frame read or written at its pass boundary once (complex64 = 8 B,
    float = 4 B).  Probe reads are shared by the batch and left out.  pairs: the inverse row
    pass writes one probe-contribution frame set per pair of slots, which the update reads."""
    nn = n * n
    xk = 4 * k if pairs else 8 * k  # probe-contribution frames per slot
    return {
        "fwd_rows": 16 * nn + 8 * k * nn,            # box gather in (exit waves and V), K frames out
        # K frames in (far field: not written back; near field: the transformed frames are stored),
        # blurred amplitude out
        "fwd_cols": (16 if near else 8) * k * nn + 4 * nn,
        "modulus_factor": 12 * nn,                   # blurred amplitude and measurement in, factor out
        "inv_cols": 16 * k * nn + 4 * nn,            # K row-transformed frames in, K frames out, factor in
        "cols_fused": 16 * k * nn + 4 * nn,          # K frames in and out, measurement in
        # K frames in, probe contributions out, box in, object numerator out
        "inv_rows_update": 8 * k * nn + xk * nn + 16 * nn,
        "obj_probe_update": xk * nn + 12 * nn,       # probe contributions in; object numerator and W gather in
    }.get(name)


def implementation_traffic(n, k, n_pos, ms_per_step, near=False, pairs=False):
    """HBM bytes of a whole iteration as the kernels move them (per_slot_bytes of every batch
    pass x positions) against the measured step time: the average rate over all kernels."""
    classes = ("fwd_rows", "fwd_cols", "modulus_factor", "inv_cols", "inv_rows_update", "obj_probe_update")
    total = sum(per_slot_bytes(c, n, k, near, pairs) for c in classes) * n_pos
    gbs = total / (ms_per_step * 1e-3) / 1e9
    return {"bytes": int(total), "achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak


def pass_model(n, k, near, positions, order, batch):
    """Algorithmic work of one iteration from the method's pass model (independent of how the
    kernels are built).  Per position: F = K n_fft 5 N^2 log2 N^2 + (30K + 60) N^2 flop
    (n_fft = 2 far field, 4 near field with (42K + 60) N^2 elementwise), compulsory bytes 12 N^2
    (pattern and box), plus per batch 16 |union of its boxes| + 16 K N^2 (object and probe read
    and written); the pass model adds one global round trip of the K frames per propagation
    direction, 32 K N^2 per position, because K 8 N^2 bytes exceed one CU's LDS."""
    nn = n * n
    lg = 2 * math.log2(n)
    n_fft = 4 if near else 2
    elem = (42 * k + 60) if near else (30 * k + 60)
    n_pos = len(positions)
    flop = n_pos * (k * n_fft * 5 * nn * lg + elem * nn)
    b_min = 12 * nn * n_pos
    for b0 in range(0, n_pos, batch):
        boxes = [positions[i] for i in order[b0:b0 + batch]]
        rows = {}
        for r, c in boxes:
            for y in range(int(r), int(r) + n):
                rows.setdefault(y, []).append((int(c), int(c) + n))
        union = 0
        for y, segs in rows.items():
            segs.sort()
            lo, hi = segs[0]
            for a, b in segs[1:]:
                if a > hi:
                    union += hi - lo
                    lo, hi = a, b
                else:
                    hi = max(hi, b)
            union += hi - lo
        b_min += 16 * union + 16 * k * nn
    b_pass = b_min + 32 * k * nn * n_pos
    return {"flop": float(flop), "bytes_min": int(b_min), "bytes_pass": int(b_pass)}


def graded(model, ms_per_step, copy_gbs):
    """t_roof / t_measured with t_roof = max(B_pass / BW, F / P_FP32), against the nominal HBM peak
    and against the device copy rate measured on this machine; and the stricter max(B_min / BW, F / P)."""
    t_meas = ms_per_step * 1e-3
    t_flop = model["flop"] / (FP32_PEAK_TFLOPS * 1e12)
    t_pass = max(model["bytes_pass"] / (HBM_PEAK_GBS * 1e9), t_flop)
    t_pass_copy = max(model["bytes_pass"] / (copy_gbs * 1e9), t_flop)
    t_min = max(model["bytes_min"] / (HBM_PEAK_GBS * 1e9), t_flop)
    return {"t_roof_ms": round(1e3 * t_pass, 4), "frac": round(t_pass / t_meas, 4),
            "frac_vs_measured_copy": round(t_pass_copy / t_meas, 4),
            "t_roof_strict_ms": round(1e3 * t_min, 4), "frac_strict": round(t_min / t_meas, 4),
            "bound": "hbm" if t_pass > t_flop else "valu", "gflop": round(model["flop"] / 1e9, 2),
            "bytes_pass_gb": round(model["bytes_pass"] / 1e9, 3), "bytes_min_gb": round(model["bytes_min"] / 1e9, 3)}


def build_workload(n_pos=None):
    import datagen
    spec = datagen.CONFIGS["far256_k4"]
    t0 = time.time()
    s = datagen.make_scan(spec, spec["seed"], n_pos=n_pos)
    return spec, s, time.time() - t0


def make_params(P, s, spec, batch):
    cp = P.default_params(n=s["n"], n_modes=s["k"], n_pos=len(s["positions"]), obj_h=s["obj0"].shape[0],
                          obj_w=s["obj0"].shape[1], geometry=s["geometry"], sigma1=spec["sigma"],
                          sigma2=spec["sigma"], batch=batch, cc_start=1, cc_end=1 << 30, alpha1=1.0,
                          alpha2=0.0, orthogonalize=1, seed=1)
    return cp


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def _oracle_batch_worker(task):
    """One oracle batch step in a worker process (the all-cores timing): returns its seconds."""
    O, Pm, sq, positions, batch, pdict = task
    import oracle as ora
    op = ora.Params(**pdict)
    t0 = time.perf_counter()
    ora.batch_step(O, Pm, sq, positions, batch, 1, op)
    return time.perf_counter() - t0


def cpu_baseline(s, spec, batch, n_batches, workers):
    """The FP64 oracle as it stands on the host cores, on the same workload: one core runs the
    first n_batches batches of iteration 1 in order; all cores run `workers` processes, each
    taking whole batches of the same iteration from the same state (the positions of one batch
    are independent work under the batched rule).  Both converted to mode-pattern updates/s."""
    import multiprocessing as mp
    import oracle as ora
    pdict = dict(n=s["n"], n_modes=s["k"], geometry=s["geometry"], fresnel_px=float(s["fresnel_px"]),
                 sigma1=spec["sigma"], sigma2=spec["sigma"], batch=batch, cc_start=1, cc_end=1 << 30, seed=1)
    op = ora.Params(**pdict)
    sq = ora.measured_amplitude(s["intensities"], op)
    order = ora.permutation(1, 1, len(s["positions"]))
    O, Pm = s["obj0"].astype(np.complex128), s["probe0"].astype(np.complex128)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.time()
    for b in range(n_batches):
        O, Pm, _, _ = ora.batch_step(O, Pm, sq, s["positions"], list(order[b * batch:(b + 1) * batch]), 1, op)
    wall = time.time() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    done = n_batches * batch * s["k"]
    nproc, model = _host_cpu()
    out = {"value": done / wall, "unit": "mode-pattern updates/s", "cores": round(cpu / wall, 1),
           "kind": "oracle", "sample": f"one core: first {n_batches} batches of {batch} positions "
           f"({n_batches * batch} of {len(s['positions'])} positions) of iteration 1 in order, {wall:.1f} s wall",
           "nproc": nproc, "cpu_model": model}
    if workers > 1:
        # each task carries only its batch's patterns (re-indexed) and the pre-iteration state
        tasks = []
        per_worker = max(1, n_batches // workers)
        for b in range(workers * per_worker):
            idx = list(order[(b % (len(order) // batch)) * batch:][:batch])
            tasks.append((s["obj0"].astype(np.complex128), s["probe0"].astype(np.complex128), sq[idx],
                          s["positions"][idx], list(range(len(idx))), pdict))
        env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
        for k in env_keep:
            os.environ[k] = "1"
        try:
            ctx = mp.get_context("spawn")
            with ctx.Pool(workers) as pool:
                pool.map(_oracle_batch_worker, tasks[:workers])  # start-up and imports off the clock
                t0 = time.time()
                secs = pool.map(_oracle_batch_worker, tasks)
                wall_all = time.time() - t0
        finally:
            for k, v in env_keep.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        done_all = len(tasks) * batch * s["k"]
        out["all_cores"] = {"value": done_all / wall_all, "unit": "mode-pattern updates/s", "cores": workers,
                            "sample": f"{len(tasks)} batches of {batch} positions of iteration 1 from the "
                                      f"initial state over {workers} single-threaded processes, {wall_all:.1f} s wall "
                                      f"({sum(secs):.1f} s of batch steps)"}
    return out


def warm_start_leg(n_iter):
    """Second metric: wall seconds to an object error on scans of the 64 x 64, 100-position
    recipe with coherence blur sigma in {0.5, 1, 2, 3} px.  The plain start (sigma 1,
    flat-phase aperture, one mode) runs each case alone; the learned start (network-predicted
    settings) runs all cases as one group with graph replay.
    * `at_1e-3`: noise-free patterns, reconstructions with the intensity blur (the data model
      of Eq. 2), error with the global scalar and the linear phase ramp removed (the ramp
      between object and probe is not determined by the data): wall seconds to 1e-3 itself.
    * `relaxed`: 1e5-count Poisson patterns, amplitude blur (Eq. 6), scalar-only error; 1e-3
      is out of reach there (noise, and the amplitude reading's drift away from the truth), so
      each case's threshold is the smallest error both single variants reach."""
    import datagen
    from paper_2406_06640_amd import evaluate as E
    net, report = E.load_warm_start()
    out = {}
    try:
        scans = []
        for i, sd in enumerate(E.SIGMA_SWEEP):
            spec = dict(datagen.CONFIGS["far64"])
            spec.update(sigma_data=sd)
            scans.append(datagen.make_scan(spec, [1005, 7, i], noise=False))
        rep = E.threshold_report(net, scans, E.SIGMA_SWEEP, n_iter, tau=1e-3, blur_domain=1, err=E.nmse_ramp)
        rep["workload"] = ("far field 64x64 frames, 10x10 raster at 8 px, object 144x144, noise-free, "
                           "sigma in {0.5,1,2,3}; intensity blur; batch 1; error with scalar and phase ramp removed")
        out["at_1e-3"] = _rounded(rep)
        scans = []
        for i, sd in enumerate(E.SIGMA_SWEEP):
            spec = dict(datagen.CONFIGS["far64"])
            spec.update(sigma_data=sd)
            scans.append(datagen.make_scan(spec, [1005, 7, i]))
        rep = E.sweep_report(net, scans, E.SIGMA_SWEEP, n_iter)
        rep["workload"] = ("far field 64x64 frames, 10x10 raster at 8 px, object 144x144, K=1, Poisson 1e5, "
                           "sigma in {0.5,1,2,3}; amplitude blur; batch 1; threshold per case = smallest "
                           "error both variants reach")
        out["relaxed"] = _rounded(rep)
    finally:
        net.close()
    out["training"] = {k: report[k] for k in ("samples", "epochs", "steps", "generation_s", "training_s",
                                              "train_samples_per_s", "val_after")}
    return out


def _rounded(obj):
    if isinstance(obj, float):
        return float(f"{obj:.5g}")
    if isinstance(obj, dict):
        return {k: _rounded(v) for k, v in obj.items()}
    if isinstance(obj, list):
        return [_rounded(v) for v in obj]
    return obj


def _time_iterations(P, torch, s, cp, steps, graph=True, autotune=True):
    """ms per iteration of one context over `steps` timed iterations (inputs in HBM, one warm-up)."""
    inten = torch.from_numpy(s["intensities"]).cuda()
    pos = torch.from_numpy(s["positions"]).cuda()
    p0 = torch.from_numpy(s["probe0"].astype(np.complex64)).cuda()
    o0 = torch.from_numpy(s["obj0"].astype(np.complex64)).cuda()
    with P.Reconstruction(cp, inten, pos, p0, o0, mem_kind=P.PTYCHO_MEM_DEVICE) as r:
        variant = r.autotune(trials=2) if autotune else None
        r.set_graph(graph)
        r.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs = r.iterate(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    return 1e3 * wall / steps, variant, float(errs[-1])


def timed_leg(P, torch, s, cp, steps, warmup, copy_gbs, near, variant=None):
    """One workload on one context: autotune, `warmup` iterations, one iteration with events
    around every launch (to find the dominant kernel), then `steps` timed iterations with
    events bound to the dominant kernel's dispatches only.  Inputs are resident in HBM before
    the timed region.  `variant` pins a launch variant instead of the autotuner's choice (for
    hardware-counter runs, under which the tuner's timings are distorted).  Returns the
    throughput, the dominant kernel's roofline and the iteration's graded fraction against
    the pass model."""
    dev = torch.device("cuda:0")
    inten = torch.from_numpy(s["intensities"]).to(dev)
    pos = torch.from_numpy(s["positions"]).to(dev)
    probe0 = torch.from_numpy(s["probe0"].astype(np.complex64)).to(dev)
    obj0 = torch.from_numpy(s["obj0"].astype(np.complex64)).to(dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    ctx = P.ptycho_init(cp, inten, pos, probe0, obj0, P.PTYCHO_MEM_DEVICE, stream)
    names = P.kernel_names()
    try:
        if variant is None:
            variant = P.ptycho_autotune(ctx, trials=3)
        else:
            P.ptycho_set_variant(ctx, variant)
        P.ptycho_iterate(ctx, warmup)
        P.ptycho_set_timing(ctx, (1 << len(names)) - 1)
        P.ptycho_iterate(ctx, 1)
        P.ptycho_set_timing(ctx, 0)
        prof = {nm: P.ptycho_kernel_time(ctx, i, reset=True) for i, nm in enumerate(names)}
        dom = max(prof, key=lambda nm: prof[nm][0])
        print("[bench] per-iteration kernel ms: " +
              ", ".join(f"{nm}={ms:.3f}({c})" for nm, (ms, c) in prof.items() if c), file=sys.stderr, flush=True)
        first_timed = P.ptycho_iteration(ctx) + 1
        P.ptycho_set_timing(ctx, 1 << names.index(dom))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs = P.ptycho_iterate(ctx, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        P.ptycho_set_timing(ctx, 0)
        dom_ms, dom_cnt = P.ptycho_kernel_time(ctx, names.index(dom), reset=True)
    finally:
        P.ptycho_destroy(ctx)
    n, k, n_pos = s["n"], s["k"], len(s["positions"])
    ms_per_step = 1e3 * wall / steps
    roof = None
    pairs = paired_rows(n, cp.batch)
    pb = per_slot_bytes(dom, n, k, near, pairs)
    if pb is not None and dom_cnt:
        # every launch of a batch kernel processes one full batch except the ragged last one
        launches_per_iter = -(-n_pos // cp.batch)
        bytes_per_launch = pb * n_pos / launches_per_iter
        avg_s = dom_ms / dom_cnt / 1e3
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom) if not near else None,
                "measured_copy_peak": round(copy_gbs, 1), "frac_of_measured_copy": round(achieved / copy_gbs, 4),
                "avg_launch_us": round(avg_s * 1e6, 2), "bytes_per_launch": int(bytes_per_launch)}
    order = P.ptycho_permutation(cp.seed, first_timed, n_pos)
    model = pass_model(n, k, near, s["positions"], order, cp.batch)
    return {"value": n_pos * k * steps / wall, "ms_per_step": ms_per_step, "roofline": roof,
            "graded": graded(model, ms_per_step, copy_gbs),
            "implementation_traffic": implementation_traffic(n, k, n_pos, ms_per_step, near, pairs),
            "kernel_ms_per_step": {nm: round(ms, 4) for nm, (ms, c) in prof.items() if c},
            "column_tile_variant": variant, "final_data_error": float(errs[-1])}


def near_field_leg(P, torch, steps, warmup, copy_gbs):
    """Near field: object 1536^2, frames 512^2, 15 x 15 positions at 60 +- 10 px, K = 8, sigma 1.5, B = 8."""
    import datagen
    spec = datagen.CONFIGS["near512_k8"]
    t0 = time.time()
    s = datagen.make_scan(spec, spec["seed"])
    gen = time.time() - t0
    print(f"[bench] near-field workload generated in {gen:.1f} s", file=sys.stderr, flush=True)
    cp = make_params(P, s, spec, spec["batch"])
    cp.geometry = 1
    cp.fresnel_px = float(s["fresnel_px"])
    leg = timed_leg(P, torch, s, cp, steps, warmup, copy_gbs, near=True)
    n_pos, k = len(s["positions"]), s["k"]
    leg.update(workload="near field, object 1536x1536, frames 512x512, 15x15 positions at 60+-10 px, K=8, "
                        "sigma 1.5, Poisson 1e6; pc-ePIE batch 8, constraint and orthogonalisation on every "
                        "iteration", positions=n_pos, modes=k, frame=s["n"], batch=cp.batch, steps=steps,
               generation_s=round(gen, 1), unit="mode-pattern updates/s")
    leg["value"] = round(leg["value"], 1)
    leg["ms_per_step"] = round(leg["ms_per_step"], 3)
    return leg


def dm_leg(P, torch, s, spec, iters, copy_gbs, batch=32):
    """The pc-DM engine (difference map with boxes 1 and 2, Sec. 4.5) on the headline
    workload: every iteration projects the object and probe from the exit waves of all
    1600 positions and runs the Fourier step of every position.  Pass model per position:
    the exit-wave state read by the object and the probe projections and read and written by
    the Fourier step (32 K N^2 bytes), the pattern and box (12 N^2), and one global round trip
    of the K frames per propagation direction (32 K N^2)."""
    dev = torch.device("cuda:0")
    n, k, n_pos = s["n"], s["k"], len(s["positions"])
    cp = make_params(P, s, spec, batch)
    cp.engine = P.PTYCHO_ENGINE_DM
    inten = torch.from_numpy(s["intensities"]).to(dev)
    pos = torch.from_numpy(s["positions"]).to(dev)
    probe0 = torch.from_numpy(s["probe0"].astype(np.complex64)).to(dev)
    obj0 = torch.from_numpy(s["obj0"].astype(np.complex64)).to(dev)
    names = P.kernel_names()
    with P.Reconstruction(cp, inten, pos, probe0, obj0, mem_kind=P.PTYCHO_MEM_DEVICE) as r:
        r.iterate(1)
        P.ptycho_set_timing(r.ctx, (1 << len(names)) - 1)
        r.iterate(1)
        P.ptycho_set_timing(r.ctx, 0)
        prof = {nm: P.ptycho_kernel_time(r.ctx, i, reset=True) for i, nm in enumerate(names)}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs = r.iterate(iters)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms = 1e3 * wall / iters
    nn = n * n
    flop = n_pos * (k * 2 * 5 * nn * 2 * math.log2(n) + (30 * k + 60) * nn)
    model = {"flop": float(flop), "bytes_min": int(n_pos * (32 * k + 12) * nn),
             "bytes_pass": int(n_pos * (64 * k + 12) * nn)}
    return {"workload": "pc-DM on the far-field 1024^2 / 256^2 / K=4 / 1600-position workload, overlap projection "
                        f"over every position, Fourier step in launches of {batch} positions, constraint every "
                        "iteration", "iterations": iters, "value": round(n_pos * k * iters / wall, 1),
            "unit": "mode-pattern updates/s", "ms_per_iteration": round(ms, 3), "graded": graded(model, ms, copy_gbs),
            "kernel_ms_per_iteration": {nm: round(v, 4) for nm, (v, c) in prof.items() if c},
            "final_data_error": float(errs[-1])}


def lsqml_leg(P, torch, s, spec, iters, copy_gbs, batch=32, lam=0.1):
    """The pc-LSQML engine (LSQML of ref. [27] with boxes 1 and 2, Sec. 3.2 and 4.1) on the
    headline workload, batch by batch as pc-ePIE.  Pass model: pc-ePIE's, plus per position the
    step normal equations' read of the K exit-wave updates, the box and the object direction
    (8 K N^2 + 16 N^2 bytes, (16 K + 40) N^2 flop), plus per batch the object direction written
    over the union of its boxes (8 |union|) and the probe direction written and read (16 K N^2)."""
    dev = torch.device("cuda:0")
    n, k, n_pos = s["n"], s["k"], len(s["positions"])
    cp = make_params(P, s, spec, batch)
    cp.engine = P.PTYCHO_ENGINE_LSQML
    cp.lsq_damping = lam
    cp.gamma_obj = cp.gamma_probe = 0.1
    inten = torch.from_numpy(s["intensities"]).to(dev)
    pos = torch.from_numpy(s["positions"]).to(dev)
    probe0 = torch.from_numpy(s["probe0"].astype(np.complex64)).to(dev)
    obj0 = torch.from_numpy(s["obj0"].astype(np.complex64)).to(dev)
    names = P.kernel_names()
    with P.Reconstruction(cp, inten, pos, probe0, obj0, mem_kind=P.PTYCHO_MEM_DEVICE) as r:
        r.iterate(1)
        P.ptycho_set_timing(r.ctx, (1 << len(names)) - 1)
        r.iterate(1)
        P.ptycho_set_timing(r.ctx, 0)
        prof = {nm: P.ptycho_kernel_time(r.ctx, i, reset=True) for i, nm in enumerate(names)}
        r.set_graph(True)
        r.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs = r.iterate(iters)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mean = r.lsq_steps()[1]
    ms = 1e3 * wall / iters
    nn = n * n
    order = P.ptycho_permutation(cp.seed, 1, n_pos)
    model = pass_model(n, k, False, s["positions"], order, batch)
    model["flop"] += float(n_pos * (16 * k + 40) * nn)
    union_total = (pass_model(n, 0, False, s["positions"], order, batch)["bytes_min"] - 12 * nn * n_pos) // 16
    extra = n_pos * (8 * k + 16) * nn + 8 * union_total + ((n_pos + batch - 1) // batch) * 16 * k * nn
    model["bytes_min"] += extra
    model["bytes_pass"] += extra
    return {"workload": "pc-LSQML on the far-field 1024^2 / 256^2 / K=4 / 1600-position workload, batch "
                        f"{batch}, damping {lam}, gammas 0.1, constraint and orthogonalisation every iteration",
            "iterations": iters, "value": round(n_pos * k * iters / wall, 1), "unit": "mode-pattern updates/s",
            "ms_per_iteration": round(ms, 3), "graded": graded(model, ms, copy_gbs),
            "kernel_ms_per_iteration": {nm: round(v, 4) for nm, (v, c) in prof.items() if c},
            "last_batch_mean_steps": [round(float(x), 4) for x in mean],
            "final_data_error": float(errs[-1])}


def c1_leg(P, torch, iters=50):
    """The 64^2-frame far-field scan (144^2 object, 10 x 10 raster at 8 px, K = 1, 1e5 counts) at
    batch size 1 -- the paper's sequential loop, 100 dependent updates per iteration -- with the
    sequential kernel (one workgroup runs the whole iteration) and with the batch passes (six
    launches per position), both replayed from a captured graph."""
    import datagen
    spec = datagen.CONFIGS["far64"]
    s = datagen.make_scan(spec, spec["seed"])
    n_pos = len(s["positions"])
    out = {"workload": "far field, object 144x144, frames 64x64, 10x10 raster at 8 px (100 positions), K=1, "
                       "sigma 1, Poisson 1e5; batch 1 (sequential updates), constraint on every iteration",
           "iterations": iters}
    for name, variant in (("sequential_kernel", P.ptycho_variant_count() - 1), ("batch_passes", 1)):
        cp = make_params(P, s, spec, 1)
        with P.Reconstruction(cp, s["intensities"], s["positions"], s["probe0"].astype(np.complex64),
                              s["obj0"].astype(np.complex64)) as r:
            r.set_variant(variant)
            r.set_graph(True)
            r.iterate(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.iterate(iters)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        out[name] = {"ms_per_iteration": round(1e3 * wall / iters, 4),
                     "us_per_position": round(1e6 * wall / iters / n_pos, 2),
                     "updates_per_s": round(n_pos * iters / wall, 1)}
    return out


def mono_leg(P, torch, s, spec, copy_gbs, k_iters=25):
    """Numerical monochromatisation by CGLS (Sec. 4.2) of the headline workload's 1600 broadband
    256^2 patterns (5 wavelengths +-2.5 %), k = 25 iterations (the paper's usual k), all patterns
    in one plan.  Algorithmic traffic per pixel and iteration: C p (read p, write q), the x / r
    update (read x, r, p, q; write x, r), C^T r (read r, write s), p = s + beta p (read s, p;
    write p): 52 bytes."""
    n = s["n"]
    scales = np.asarray(spec["wavelengths"], dtype=np.float32)
    weights = np.ones_like(scales)
    b = torch.from_numpy(s["intensities"]).cuda()
    out = torch.empty_like(b)
    n_pat = b.shape[0]
    with P.Monochromatiser(n, n_pat, scales, weights) as mc:
        mc.run(b, out, 2, residuals=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = mc.run(b, out, k_iters, residuals=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    nbytes = 52.0 * n * n * n_pat * k_iters
    gbs = nbytes / wall / 1e9
    drop = res[:, -1] / np.maximum(res[:, 0], 1e-30)
    return {"workload": f"{n_pat} broadband patterns of {n}x{n} (5 wavelengths +-2.5 %), CGLS k={k_iters}",
            "wall_s": round(wall, 4), "patterns_per_s": round(n_pat / wall, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": int(nbytes)},
            "residual_ratio_median": float(np.median(drop))}


def group_leg(P, torch, iters, copy_gbs, n_cases=64):
    """The 64-case batched workload (N in {64,128,192,256}, 100-2500 positions, 1-8 modes, batch
    32, seeds [1004, i]; patterns made on the GPU) advanced as one group with graph replay:
    throughput, and the pass-model roofline per case and in aggregate (the sum over cases of
    t_roof against the group's measured time per iteration)."""
    import datagen
    from datagen import gpu_synth
    t0 = time.time()
    cases = []
    for i in range(n_cases):
        sp = datagen.random_case_spec(i)
        cases.append((sp, gpu_synth.make_scan(sp, sp["seed_key"])))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    print(f"[bench] {n_cases}-case workload generated in {gen_s:.1f} s", file=sys.stderr, flush=True)
    recs = []
    for sp, sc in cases:
        h, w = sc["obj0"].shape
        cp = P.default_params(n=sc["n"], n_modes=sc["k"], n_pos=len(sc["positions"]), obj_h=h, obj_w=w,
                              sigma1=sp["sigma"], sigma2=sp["sigma"], batch=sp["batch"], seed=1)
        cp.cc_start, cp.cc_end = 1, 0
        pos = torch.from_numpy(sc["positions"]).cuda()
        p0 = torch.from_numpy(sc["probe0"].astype(np.complex64)).cuda()
        o0 = torch.from_numpy(sc["obj0"].astype(np.complex64)).cuda()
        recs.append(P.Reconstruction(cp, sc["intensities_dev"], pos, p0, o0, mem_kind=P.PTYCHO_MEM_DEVICE))
    try:
        with P.Group(recs) as g:
            g.set_graph(True)
            g.iterate(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.iterate(iters)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
    finally:
        for r in recs:
            r.close()
    ms = 1e3 * wall / iters
    updates = sum(len(sc["positions"]) * sc["k"] for _, sc in cases)
    per_case, tot = [], {"flop": 0.0, "bytes_min": 0, "bytes_pass": 0}
    for (sp, sc) in cases:
        order = P.ptycho_permutation(1, 2, len(sc["positions"]))
        m = pass_model(sc["n"], sc["k"], False, sc["positions"], order, sp["batch"])
        for key in tot:
            tot[key] += m[key]
        t_roof = max(m["bytes_pass"] / (HBM_PEAK_GBS * 1e9), m["flop"] / (FP32_PEAK_TFLOPS * 1e12))
        per_case.append({"n": sc["n"], "k": sc["k"], "positions": len(sc["positions"]),
                         "t_roof_ms": round(1e3 * t_roof, 4), "gflop": round(m["flop"] / 1e9, 3),
                         "bytes_pass_gb": round(m["bytes_pass"] / 1e9, 4)})
    return {"workload": f"{n_cases} far-field cases, N in {{64,128,192,256}}, 100-2500 positions, K 1-8, "
                        "batch 32, Poisson 1e5, sigma 1; seeds [1004, i]; one group, graph replay",
            "iterations": iters, "mode_pattern_updates_per_iteration": updates,
            "value": round(updates * iters / wall, 1), "unit": "mode-pattern updates/s",
            "ms_per_iteration": round(ms, 3), "graded": graded(tot, ms, copy_gbs),
            "per_case": per_case, "generation_s": round(gen_s, 1)}


# The paper's own QPT scans (Table 1: 100 points, 1024^2 patterns, 0.02 mm steps over 2.71 um
# (far) or 6.5 um (near) object pixels; near field 19.9 mm at 514.5 nm with 6.5 um pixels, so
# F_px = 6.5^2 / (0.5145 * 19900)) and their per-iteration pc-ePIE times on a TITAN Xp (captions of
# Figs. 4 and 3).
PAPER_FRAME = 1024
PAPER_SCAN_SIDE = 10
PAPER_SHAPES = (("far", 0, 7, 0.0, 452.2), ("near", 1, 3, 4.13e-3, 640.0))  # name, geometry, step, F_px, ms


def paper_shapes_leg(steps=5):
    """The paper's scans (100 patterns of 1024^2, one mode): far field at a 7 px step, near field at
    3 px with F_px = 4.13e-3; sequential updates (batch 1, as the paper's loop) and batch 10."""
    import torch
    import datagen
    import paper_2406_06640_amd as P
    out = {}
    for name, geometry, step, fresnel_px, paper_ms in PAPER_SHAPES:
        n = PAPER_FRAME
        extent = (PAPER_SCAN_SIDE - 1) * step + n + 2
        side = int(np.ceil(extent / 16.0) * 16)
        spec = dict(datagen.CONFIGS["far64"])
        spec.update(geometry=geometry, obj=(side, side), n=n, n_side=PAPER_SCAN_SIDE, step=step, jitter=1, k=1,
                    powers=(1.0,), radius=n // 4, defocus=1.0 if geometry == 0 else 0.0, sigma_data=1.0,
                    counts=1e6, fresnel_px=fresnel_px, sigma=1.0, batch=1)
        t0 = time.time()
        s = datagen.make_scan(spec, [1006, geometry])
        gen = time.time() - t0
        row = {"generation_s": round(gen, 1), "paper_ms_per_iteration": paper_ms}
        for b in (1, 10):
            cp = make_params(P, s, spec, b)
            cp.geometry = geometry
            cp.fresnel_px = float(spec["fresnel_px"])
            cp.sigma1 = cp.sigma2 = 1.0
            ms, variant, _ = _time_iterations(P, torch, s, cp, steps)
            row[f"ms_per_iteration_batch{b}"] = round(ms, 3)
        row["speedup_vs_paper_batch1"] = round(paper_ms / row["ms_per_iteration_batch1"], 1)
        out[name] = row
    out["workload"] = ("100 patterns of 1024x1024 (10x10 raster), one mode, sigma 1, 11x11 blur, constraint on; "
                       "far field step 7 px, near field step 3 px with F_px 4.13e-3; the paper's times are "
                       "for a TITAN Xp (ePIE-family code, precision not stated)")
    return out


def batched_leg(iters):
    """The 64-case batched workload (N in {64,128,192,256}, 100-2500 positions, 1-8 modes, batch 32,
    seeds [1004, i]; patterns made on the GPU): every case alone (autotuned, graph replay) against
    all cases as one group (graph replay), same final states required bitwise; and the BF16
    matrix-core DFT path on the cases whose N it supports, with its object error against the
    FP32 FFT path after the same iterations."""
    import torch
    import datagen
    from datagen import gpu_synth
    import paper_2406_06640_amd as P
    t0 = time.time()
    cases = []
    for i in range(64):
        sp = datagen.random_case_spec(i)
        cases.append((sp, gpu_synth.make_scan(sp, sp["seed_key"])))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    print(f"[bench] 64-case workload generated in {gen_s:.1f} s", file=sys.stderr, flush=True)

    def make(sp, s, dft=False):
        h, w = s["obj0"].shape
        cp = P.default_params(n=s["n"], n_modes=s["k"], n_pos=len(s["positions"]), obj_h=h, obj_w=w,
                              sigma1=sp["sigma"], sigma2=sp["sigma"], batch=sp["batch"], seed=1,
                              dft_bf16=1 if dft else 0)
        cp.cc_start, cp.cc_end = 1, 0
        pos = torch.from_numpy(s["positions"]).cuda()
        p0 = torch.from_numpy(s["probe0"].astype(np.complex64)).cuda()
        o0 = torch.from_numpy(s["obj0"].astype(np.complex64)).cuda()
        return P.Reconstruction(cp, s["intensities_dev"], pos, p0, o0, mem_kind=P.PTYCHO_MEM_DEVICE)

    updates = sum(len(s["positions"]) * s["k"] for _, s in cases)
    singles = [make(sp, s) for sp, s in cases]
    variants = [r.autotune(trials=2) for r in singles]
    for r in singles:
        r.set_graph(True)
        r.iterate(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in singles:
        r.iterate(iters)
    torch.cuda.synchronize()
    wall_single = time.perf_counter() - t0
    grouped = [make(sp, s) for sp, s in cases]
    with P.Group(grouped) as g:
        g.set_graph(True)
        g.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.iterate(iters)
        torch.cuda.synchronize()
        wall_group = time.perf_counter() - t0
    same = all(np.array_equal(a.object(), b.object()) and np.array_equal(a.probe(), b.probe())
               for a, b in zip(singles, grouped))
    for r in grouped:
        r.close()
    dft_rows, wall_dft, wall_fft_sub, upd_sub = [], 0.0, 0.0, 0
    for (sp, s), ref in zip(cases, singles):
        if s["n"] not in (64, 128, 192, 256):
            continue
        with make(sp, s, dft=True) as r:
            r.iterate(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.iterate(iters)
            torch.cuda.synchronize()
            wall_dft += time.perf_counter() - t0
            o = r.object().astype(np.complex128)
        o_ref = ref.object().astype(np.complex128)
        dft_rows.append({"n": s["n"], "k": s["k"], "positions": len(s["positions"]),
                         "object_rel_l2_vs_fp32": float(np.linalg.norm(o - o_ref) / np.linalg.norm(o_ref))})
        upd_sub += len(s["positions"]) * s["k"]
    # the FP32 path on the same subset (eager launches like the DFT runs), for the comparison
    for (sp, s), r in zip(cases, singles):
        if s["n"] in (64, 128, 192, 256):
            r.set_graph(False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.iterate(iters)
            torch.cuda.synchronize()
            wall_fft_sub += time.perf_counter() - t0
    for r in singles:
        r.close()
    errs = [row["object_rel_l2_vs_fp32"] for row in dft_rows]
    return {
        "workload": "64 far-field cases, N in {64,128,192,256}, 100-2500 positions, K 1-8, batch 32, "
                    "Poisson 1e5, sigma 1; seeds [1004, i]",
        "iterations": iters, "mode_pattern_updates_per_iteration": updates, "generation_s": round(gen_s, 2),
        "one_by_one": {"wall_s": round(wall_single, 4), "updates_per_s": round(updates * iters / wall_single, 1)},
        "group": {"wall_s": round(wall_group, 4), "updates_per_s": round(updates * iters / wall_group, 1),
                  "bitwise_equal_to_one_by_one": bool(same)},
        "autotuned_variants": variants,
        "dft_bf16": {"cases": len(dft_rows), "wall_s": round(wall_dft, 4),
                     "updates_per_s": round(upd_sub * iters / wall_dft, 1) if wall_dft else None,
                     "fp32_fft_updates_per_s_same_cases": round(upd_sub * iters / wall_fft_sub, 1)
                     if wall_fft_sub else None,
                     "object_rel_l2_vs_fp32_max": max(errs) if errs else None,
                     "object_rel_l2_vs_fp32_median": float(np.median(errs)) if errs else None,
                     "per_case": dft_rows},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-batches", type=int, default=40)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-cores oracle timing (capped by the host's CPU count)")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the time-to-error comparison of the plain and the learned + batched start")
    ap.add_argument("--warm-start-iterations", type=int, default=50)
    ap.add_argument("--no-near-field", action="store_true",
                    help="skip the near-field 1536^2 / 512^2 / K=8 workload")
    ap.add_argument("--near-field-steps", type=int, default=5)
    ap.add_argument("--no-group", action="store_true", help="skip the 64-case workload as one group")
    ap.add_argument("--no-dm", action="store_true", help="skip the pc-DM engine leg")
    ap.add_argument("--no-c1", action="store_true", help="skip the 64^2-frame batch-1 leg")
    ap.add_argument("--no-mono", action="store_true", help="skip the CGLS monochromatisation leg")
    ap.add_argument("--no-lsqml", action="store_true", help="skip the pc-LSQML engine leg")
    ap.add_argument("--lsqml-iterations", type=int, default=3)
    ap.add_argument("--dm-iterations", type=int, default=3)
    ap.add_argument("--group-iterations", type=int, default=3)
    ap.add_argument("--batched", action="store_true",
                    help="also run the 64-case batched workload's full comparison: group vs the cases one by "
                         "one, and the BF16 matrix-core DFT path")
    ap.add_argument("--batched-iterations", type=int, default=3)
    ap.add_argument("--paper-shapes", action="store_true",
                    help="also time the paper's own scan shapes (100 patterns of 1024^2, one mode, far and near "
                         "field) for comparison with its per-iteration times")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 256 MiB device-to-device tensor copy (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--only-headline", action="store_true", help="time the headline workload only (profiling)")
    ap.add_argument("--variant", type=int, default=None,
                    help="launch variant of the headline workload instead of the autotuner's choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2406_06640_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbs = copy_bandwidth(torch, dev)
    spec, s, gen_s = build_workload()
    print(f"[bench] workload generated in {gen_s:.1f} s", file=sys.stderr, flush=True)
    n, k, n_pos = s["n"], s["k"], len(s["positions"])
    cp = make_params(P, s, spec, args.batch)
    leg = timed_leg(P, torch, s, cp, args.steps, args.warmup, copy_gbs, near=False, variant=args.variant)
    out = {
        "metric": "mode-pattern updates/s",
        "value": round(leg["value"], 1),
        "unit": "mode-pattern updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(leg["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded forward model; see datagen/)",
        "config": {"workload": "far field, object 1024x1024, frames 256x256, 40x40 raster at 16 px "
                               "(1600 positions), K=4 modes, 5 wavelengths +-2.5%, sigma=2, Poisson 1e6; "
                               f"pc-ePIE batch {args.batch}, 11x11 blur, complex constraint and "
                               "orthogonalisation on every timed iteration",
                   "positions": n_pos, "modes": k, "frame": n, "batch": args.batch,
                   "column_tile_variant": leg["column_tile_variant"]},
        "roofline": leg["roofline"],
        "graded": leg["graded"],
        "implementation_traffic": leg["implementation_traffic"],
        "kernel_ms_per_step": leg["kernel_ms_per_step"],
        "final_data_error": leg["final_data_error"],
    }
    if not args.only_headline:
        if not args.no_near_field:
            print("[bench] near-field workload", file=sys.stderr, flush=True)
            out["near_field"] = near_field_leg(P, torch, args.near_field_steps, args.warmup, copy_gbs)
        if not args.no_c1:
            print("[bench] 64^2 scan at batch 1 (sequential kernel vs batch passes)", file=sys.stderr, flush=True)
            out["c1_batch1"] = c1_leg(P, torch)
        if not args.no_dm:
            print("[bench] pc-DM engine on the headline workload", file=sys.stderr, flush=True)
            out["dm"] = dm_leg(P, torch, s, spec, args.dm_iterations, copy_gbs)
        if not args.no_lsqml:
            print("[bench] pc-LSQML engine on the headline workload", file=sys.stderr, flush=True)
            out["lsqml"] = lsqml_leg(P, torch, s, spec, args.lsqml_iterations, copy_gbs)
        if not args.no_mono:
            print("[bench] CGLS monochromatisation of the headline patterns", file=sys.stderr, flush=True)
            out["monochromatisation"] = mono_leg(P, torch, s, spec, copy_gbs)
        if not args.no_group:
            print("[bench] 64-case workload as one group", file=sys.stderr, flush=True)
            out["group"] = group_leg(P, torch, args.group_iterations, copy_gbs)
        if not args.no_warm_start:
            print("[bench] time to object error, plain vs learned + batched", file=sys.stderr, flush=True)
            out["time_to_nmse"] = warm_start_leg(args.warm_start_iterations)
        if args.paper_shapes:
            print("[bench] paper-shape scans", file=sys.stderr, flush=True)
            out["paper_shapes"] = paper_shapes_leg()
        if args.batched:
            print("[bench] 64-case batched workload, full comparison", file=sys.stderr, flush=True)
            out["batched"] = batched_leg(args.batched_iterations)
        if not args.no_cpu_baseline:
            print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
            workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
            out["cpu_baseline"] = cpu_baseline(s, spec, args.batch, args.cpu_batches, workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
