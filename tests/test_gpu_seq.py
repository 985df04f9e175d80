"""GPU parity of the sequential kernel (batch size 1, far-field frames of side
16-64: one workgroup runs a whole iteration of Fig. 1's loop) against the FP64
oracle, against the batch passes, and as groups.

Bar: per iteration from a shared state, relative L2 <= 1e-5 for the object (on
the union of the boxes), the probe and E_t; the worst element within 1e-4 of
the peak.  An iteration here is 16-100 dependent updates, each carrying the
previous one's rounding, which the per-iteration bar absorbs at these sizes.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as ora
from parity_util import inf_rel, make_case, params_pair, probe_metrics, rel_l2, state32, union_of_boxes

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_INF = 1e-4


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _orders(seed, n_iter, n_pos):
    return np.stack([ora.permutation(seed, t, n_pos) for t in range(1, n_iter + 1)]).astype(np.int32)


CASES = {
    "c1_n64_k1_window": (dict(n=64, obj=(144, 144), n_side=10, step=8, radius=16, seed=1001),
                         dict(batch=1, cc_start=2, cc_end=3), 3),
    "n32_k2_intensity_gammas": (dict(n=32, k=2, obj=(80, 80), n_side=5, step=8, seed=91),
                                dict(batch=1, blur_domain=1, gamma_obj=0.6, gamma_probe=0.8, eps=1e-3,
                                     sigma1=0.7, sigma2=1.3, kernel_size=9), 2),
    "n48_k3_radix3_frozen_probe": (dict(n=48, k=3, obj=(96, 96), n_side=4, step=12, radius=12, seed=92),
                                   dict(batch=1, probe_update_start=2, cc_start=1, cc_end=1), 2),
    "n16_k1_single_stage": (dict(n=16, obj=(48, 48), n_side=4, step=6, radius=5, seed=93),
                            dict(batch=1, kernel_size=5), 2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_seq_iteration_parity(name):
    import paper_2406_06640_amd as P
    ckw, pkw, n_iter = CASES[name]
    s = make_case(**ckw)
    if s["k"] > 1:
        s["probe0"] = s["probe_true"]  # distinct mode powers
    cp, op = params_pair(s, **pkw)
    _announce(f"seq {name} n={cp.n} K={cp.n_modes} positions={len(s['positions'])}")
    orders = _orders(5, n_iter, len(s["positions"]))
    roi = union_of_boxes(s["positions"], s["n"], s["obj0"].shape)
    o32, p32 = state32(s)
    sq = ora.measured_amplitude(s["intensities"], op)
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as rec:
        assert rec.autotune() == P.ptycho_variant_count() - 1  # the sequential kernel
        st = ora.State(O=o32.astype(np.complex128), P=p32.astype(np.complex128))
        for it in range(n_iter):
            o_r, p_r = st.O.astype(np.complex64), st.P.astype(np.complex64)
            rec.set_state(o_r, p_r, it)
            st = ora.State(O=o_r.astype(np.complex128), P=p_r.astype(np.complex128), t=it)
            e_g = rec.iterate(1, orders[it:it + 1])
            st, e_o = ora.iterate(st, None, s["positions"], op, 1, orders=orders[it:it + 1], sqrt_I=sq)
            og, pg = rec.object(), rec.probe()
            r = dict(O=rel_l2(og[roi], st.O[roi]), O_inf=inf_rel(og[roi], st.O[roi]), P=rel_l2(pg, st.P),
                     P_inf=inf_rel(pg, st.P), err=abs(float(e_g[0]) - e_o[0]) / abs(e_o[0]))
            r.update(probe_metrics(pg, st.P))
            print(it + 1, {k: f"{v:.2e}" for k, v in r.items()}, flush=True)
            for key in ("O", "P", "err", "sum_p2", "eig"):
                assert r[key] <= TOL, (key, r)
            for key in ("O_inf", "P_inf"):
                assert r[key] <= TOL_INF, (key, r)
            np.testing.assert_array_equal(og[~roi], o_r[~roi])


def test_seq_matches_batch_passes_and_is_deterministic():
    """The sequential kernel and the batch passes (variant 1) run the same method: after two
    iterations of the C1 workload they agree to FP32 rounding; two sequential runs agree bitwise."""
    import paper_2406_06640_amd as P
    s = make_case(n=64, obj=(144, 144), n_side=10, step=8, radius=16, seed=1001)
    cp, _ = params_pair(s, batch=1, cc_start=1, cc_end=2)
    _announce("seq vs batch passes, C1")
    o32, p32 = state32(s)
    orders = _orders(7, 2, len(s["positions"]))
    out = []
    for variant in (None, 1, None):
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            if variant is not None:
                r.set_variant(variant)
            e = r.iterate(2, orders)
            out.append((r.object(), r.probe(), e))
    for a, b in zip(out[0], out[2]):
        np.testing.assert_array_equal(a, b)
    print({"O": rel_l2(out[0][0], out[1][0]), "P": rel_l2(out[0][1], out[1][1])}, flush=True)
    assert rel_l2(out[0][0], out[1][0]) <= 1e-5
    assert rel_l2(out[0][1], out[1][1]) <= 1e-5
    assert np.max(np.abs(out[0][2] - out[1][2]) / out[1][2]) <= 1e-5


def test_seq_group_matches_single_runs():
    """Sequential cases in a group (one workgroup each, one launch) beside a batch-pass case:
    every case bitwise equal to its single run, eager and graph-replayed."""
    import paper_2406_06640_amd as P
    specs = [(dict(n=64, obj=(144, 144), n_side=10, step=8, radius=16, seed=94), dict(batch=1, seed=3)),
             (dict(n=64, k=2, obj=(128, 128), n_side=6, step=12, radius=16, seed=95), dict(batch=1, seed=4)),
             (dict(n=32, obj=(72, 72), n_side=4, step=8, seed=96), dict(batch=1, seed=5, cc_start=1, cc_end=1)),
             (dict(n=64, obj=(128, 128), n_side=5, step=12, radius=16, seed=97), dict(batch=4, seed=6))]
    _announce("group: three sequential cases and one batch-pass case")
    made = []
    for ckw, pkw in specs:
        s = make_case(**ckw)
        cp, _ = params_pair(s, **pkw)
        made.append((s, cp))
    singles = []
    for s, cp in made:
        o32, p32 = state32(s)
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            e = r.iterate(3)
            singles.append((r.object(), r.probe(), e))
    for graph in (False, True):
        recs = []
        try:
            for s, cp in made:
                o32, p32 = state32(s)
                recs.append(P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32))
            with P.Group(recs) as g:
                g.set_graph(graph)
                errs = np.concatenate([g.iterate(2), g.iterate(1)], axis=1)
            for i, r in enumerate(recs):
                np.testing.assert_array_equal(r.object(), singles[i][0], err_msg=f"case {i} object")
                np.testing.assert_array_equal(r.probe(), singles[i][1], err_msg=f"case {i} probe")
                np.testing.assert_array_equal(errs[i], singles[i][2], err_msg=f"case {i} error")
        finally:
            for r in recs:
                r.close()
