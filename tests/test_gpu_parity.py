"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bar: relative L2 <= 1e-5 for the FP32 exit waves (psi, psi') and the updates
(object/probe numerators and weights, the updated object and probe), per batch
step from an identical state and per iteration.  The modulus factor is a
ratio whose dim-pixel entries inherit the FFT's absolute rounding; it is held
to 1e-4.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as ora
from parity_util import gpu_step, inf_rel, make_case, oracle_step, params_pair, rel_l2, state32

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_FACTOR = 1e-4
# worst single element against the reference's peak magnitude: FP32 rounding of one
# element through ~20 transform stages is ~1e-6 of the peak; dim pixels of psi' carry
# the modulus factor's relative error, so the bar is set an order above that
TOL_INF = 1e-4


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _compare_step(gc, oc, cp, check_probe=True, tol=TOL):
    out = {}
    out["psi"] = rel_l2(gc["psi"], np.stack(oc["psi"]))
    out["psi_new"] = rel_l2(gc["psi_new"], np.stack(oc["psi_new"]))
    out["factor"] = rel_l2(gc["factor"], np.stack(oc["factor"]))
    out["n_obj"] = rel_l2(gc["n_obj"], oc["n_o"])
    out["w_obj"] = rel_l2(gc["w_obj"], oc["w"])
    m = oc["mask"]  # union of the batch's boxes: the only pixels the step changes
    out["O"] = rel_l2(gc["O"][m], oc["O"][m])
    out["P"] = rel_l2(gc["P"], oc["P"])
    if check_probe:
        out["n_probe"] = rel_l2(gc["n_probe"], oc["n_p"])
        out["v_probe"] = rel_l2(gc["v_probe"], oc["v"])
    inf = {"psi_new": inf_rel(gc["psi_new"], np.stack(oc["psi_new"])), "n_obj": inf_rel(gc["n_obj"], oc["n_o"]),
           "O": inf_rel(gc["O"][m], oc["O"][m]), "P": inf_rel(gc["P"], oc["P"])}
    if check_probe:
        inf["n_probe"] = inf_rel(gc["n_probe"], oc["n_p"])
    print({k: f"{v:.2e}" for k, v in out.items()}, "worst element:", {k: f"{v:.1e}" for k, v in inf.items()},
          flush=True)
    for k, v in out.items():
        lim = TOL_FACTOR if k == "factor" else tol
        assert v <= lim, f"{k}: relative L2 {v:.3e} > {lim:g}"
    for k, v in inf.items():
        assert v <= max(TOL_INF, 10 * tol), f"{k}: worst element {v:.3e} of the peak > {TOL_INF:g}"
    # pixels outside the batch's boxes keep their values exactly
    np.testing.assert_array_equal(gc["O"][~m], oc["O"][~m].astype(np.complex64))
    return out


STEP_CASES = {
    # name: (make_case kwargs, params kwargs, batch indices, t)
    "far_n64_k1_b1": (dict(n=64, obj=(144, 144), n_side=10, step=8, radius=16), dict(batch=1), [37], 1),
    "far_n32_k2_ragged": (dict(n=32, k=2, obj=(80, 80), n_side=5, step=8),
                          dict(batch=5, sigma1=0.8, sigma2=1.3, kernel_size=7), [3, 17, 9], 1),
    "far_n192_k3_radix3": (dict(n=192, k=3, obj=(260, 260), n_side=3, step=24, radius=40),
                           dict(batch=2), [4, 1], 1),
    "near_n64_k2": (dict(n=64, k=2, geometry=1, obj=(128, 128), n_side=4, step=16, radius=16),
                    dict(batch=4, sigma1=1.5, sigma2=1.5), [0, 5, 10, 15], 1),
    "far_intensity_gammas": (dict(n=48, k=2, obj=(96, 96), n_side=4, step=10),
                             dict(batch=4, blur_domain=1, gamma_obj=0.5, gamma_probe=0.7, eps=1e-3),
                             [2, 7, 11, 13], 2),
    "far_constraint_window": (dict(n=32, k=1, obj=(72, 72), n_side=4, step=8),
                              dict(batch=3, cc_start=1, cc_end=5, alpha1=0.6, alpha2=0.3), [0, 6, 12], 2),
    "probe_frozen": (dict(n=24, k=1, obj=(64, 64), n_side=4, step=8),
                     dict(batch=2, probe_update_start=5), [1, 2], 3),
    "far_n128_k4": (dict(n=128, k=4, obj=(200, 200), n_side=3, step=24, radius=30),
                    dict(batch=3), [0, 4, 8], 1),
    # odd batches at sizes with the paired inverse row pass: the last pair has one slot
    "far_n256_k2_odd_pairs": (dict(n=256, k=2, obj=(320, 320), n_side=3, step=24, radius=48),
                              dict(batch=5, sigma1=2.0, sigma2=2.0), [8, 0, 4, 2, 6], 1),
    "near_n512_k2_odd_pairs": (dict(n=512, k=2, geometry=1, obj=(576, 576), n_side=2, step=48, radius=100),
                               dict(batch=3, sigma1=1.5, sigma2=1.5), [3, 0, 1], 1),
}


@pytest.mark.parametrize("name", list(STEP_CASES))
def test_batch_step_parity(name):
    ckw, pkw, idx, t = STEP_CASES[name]
    s = make_case(**ckw)
    cp, op = params_pair(s, **pkw)
    _announce(f"step {name} n={cp.n} K={cp.n_modes} B={len(idx)} t={t} geometry={cp.geometry}")
    gc, o32, p32 = gpu_step(s, cp, idx, t)
    oc = oracle_step(s, op, idx, t, o32, p32)
    _compare_step(gc, oc, cp, check_probe=t >= op.probe_update_start)
    if t < op.probe_update_start:
        np.testing.assert_array_equal(gc["P"], p32)


def _orders(seed, t0, n_iter, n_pos):
    return np.stack([ora.permutation(seed, t0 + i + 1, n_pos) for i in range(n_iter)]).astype(np.int32)


def _iterate_both(s, cp, op, n_iter, orders, chained=False):
    """Per-iteration parity: before each iteration the GPU state is set to the
    oracle's state (rounded to complex64) so both run the iteration from the
    same state; with chained=True the two runs continue independently and the
    accumulated drift is measured instead."""
    import paper_2406_06640_amd as P
    o32, p32 = state32(s)
    rec = P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32)
    st = ora.State(O=o32.astype(np.complex128), P=p32.astype(np.complex128))
    sq = ora.measured_amplitude(s["intensities"], op)
    res = []
    try:
        for it in range(n_iter):
            if not chained:
                o_r, p_r = st.O.astype(np.complex64), st.P.astype(np.complex64)
                rec.set_state(o_r, p_r, it)
                st = ora.State(O=o_r.astype(np.complex128), P=p_r.astype(np.complex128), t=it)
            e_g = rec.iterate(1, orders[it:it + 1])
            st, e_o = ora.iterate(st, None, s["positions"], op, 1, orders=orders[it:it + 1], sqrt_I=sq)
            res.append(dict(O=rel_l2(rec.object(), st.O), P=rel_l2(rec.probe(), st.P),
                            err=abs(float(e_g[0]) - e_o[0]) / abs(e_o[0])))
            print(it + 1, "chained" if chained else "", {k: f"{v:.2e}" for k, v in res[-1].items()}, flush=True)
    finally:
        rec.close()
    return res


@pytest.mark.parametrize("batch", [1, 10])
def test_iteration_parity_c1(batch):
    """Config-1 workload (far field, 64^2 frames, 10x10 raster, K = 1), constraint
    window in iterations 2-3: every iteration from a shared state within 1e-5."""
    s = make_case(n=64, obj=(144, 144), n_side=10, step=8, radius=16, seed=1001)
    cp, op = params_pair(s, batch=batch, cc_start=2, cc_end=3)
    _announce(f"iterations c1 batch={batch}")
    res = _iterate_both(s, cp, op, 3, _orders(5, 0, 3, len(s["positions"])))
    for r in res:
        assert r["O"] <= TOL and r["P"] <= TOL and r["err"] <= TOL, r


def test_chained_drift_c1():
    """Three chained iterations of 100 sequential (B = 1) updates each: rounding
    differences of ~1e-7 per step are amplified by the iteration itself, so the
    drift is held to a looser 1e-4 and reported."""
    s = make_case(n=64, obj=(144, 144), n_side=10, step=8, radius=16, seed=1001)
    cp, op = params_pair(s, batch=1)
    _announce("chained drift c1 batch=1")
    res = _iterate_both(s, cp, op, 3, _orders(5, 0, 3, len(s["positions"])), chained=True)
    for r in res:
        assert r["O"] <= 1e-4 and r["P"] <= 1e-4 and r["err"] <= 1e-4, r


def test_iteration_parity_near_modes():
    s = make_case(n=64, k=3, geometry=1, obj=(128, 128), n_side=4, step=16, radius=16, seed=3)
    cp, op = params_pair(s, batch=4, sigma1=1.5, sigma2=1.5)
    _announce("iterations near K=3 ortho")
    res = _iterate_both(s, cp, op, 2, _orders(9, 0, 2, len(s["positions"])))
    for r in res:
        assert r["O"] <= TOL and r["err"] <= TOL, r
        # modes are defined up to unitary mixing among near-degenerate eigenvalues;
        # the probe as a whole still matches mode by mode for these well-separated powers
        assert r["P"] <= TOL, r


def test_determinism_and_resume():
    import paper_2406_06640_amd as P
    s = make_case(n=32, k=2, obj=(80, 80), n_side=5, step=8, seed=21)
    cp, _ = params_pair(s, batch=4, cc_start=1, cc_end=2)
    _announce("determinism/resume n=32 K=2")
    o32, p32 = state32(s)
    orders = _orders(2, 0, 3, len(s["positions"]))
    runs = []
    for _ in range(2):
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            e = r.iterate(3, orders)
            runs.append((r.object(), r.probe(), e))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    np.testing.assert_array_equal(runs[0][2], runs[1][2])
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        r.iterate(2, orders[:2])
        o2, p2 = r.object(), r.probe()
        assert r.iteration == 2
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        r.set_state(o2, p2, 2)
        e3 = r.iterate(1, orders[2:3])
        np.testing.assert_array_equal(r.object(), runs[0][0])
        np.testing.assert_array_equal(r.probe(), runs[0][1])
        np.testing.assert_array_equal(e3, runs[0][2][2:3])


def test_split_calls_match_one_call():
    """Iterations spread over several calls (eager and graph-replayed) give bitwise the
    result of one call: 25 positions in batches of 4 (an odd number of batches per
    iteration), the probe frozen for the first two iterations, a constraint window."""
    import paper_2406_06640_amd as P
    s = make_case(n=32, k=2, obj=(80, 80), n_side=5, step=8, seed=23)
    cp, _ = params_pair(s, batch=4, probe_update_start=3, cc_start=2, cc_end=3)
    _announce("split calls n=32 K=2 odd batch count")
    o32, p32 = state32(s)
    orders = _orders(7, 0, 5, len(s["positions"]))
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        e_all = r.iterate(5, orders)
        ref = (r.object(), r.probe())
    for graph, cuts in ((False, (1, 2, 3, 4)), (True, (2,)), (True, (1, 3))):
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            r.set_graph(graph)
            errs, lo = [], 0
            for hi in list(cuts) + [5]:
                errs.append(r.iterate(hi - lo, orders[lo:hi]))
                lo = hi
            np.testing.assert_array_equal(r.object(), ref[0])
            np.testing.assert_array_equal(r.probe(), ref[1])
            np.testing.assert_array_equal(np.concatenate(errs), e_all)


def test_library_order_generator_matches_explicit():
    import paper_2406_06640_amd as P
    s = make_case(n=32, obj=(72, 72), n_side=4, step=8, seed=4)
    cp, _ = params_pair(s, batch=2, seed=99)
    _announce("generator order")
    o32, p32 = state32(s)
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        r.iterate(2)
        a = r.object()
    orders = _orders(99, 0, 2, len(s["positions"]))
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        r.iterate(2, orders)
        np.testing.assert_array_equal(r.object(), a)


@pytest.mark.parametrize("cfg,variant", [("far256_k4", None), ("far256_k4", 10), ("near512_k8", None),
                                         ("near512_k8", 10)])
def test_full_size_batch_step(cfg, variant):
    """One batch at the full frame size and batch size of the 1024^2 far-field
    (256^2 frames, K = 4, B = 32, 5-wavelength data) and 1536^2 near-field
    (512^2 frames, K = 8, B = 8) workloads, constraint window on; in the default
    launch configuration and in variant 10 (mode-parallel first row pass and
    inverse column pass), the one the autotuner picks for both in the benchmark."""
    import datagen
    spec = datagen.CONFIGS[cfg]
    B = spec["batch"]
    s = datagen.make_scan(spec, spec["seed"], n_pos=2 * B)
    cp, op = params_pair(s, batch=B, cc_start=1, cc_end=10)
    idx = list(range(1, 2 * B, 2))
    _announce(f"full-size step {cfg} n={cp.n} K={cp.n_modes} B={B} variant={variant}")
    gc, o32, p32 = gpu_step(s, cp, idx, 1, variant=variant)
    oc = oracle_step(s, op, idx, 1, o32, p32)
    _compare_step(gc, oc, cp)
