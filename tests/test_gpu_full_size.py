"""Per-iteration GPU parity at the full frame and batch sizes of the two large
workloads, and of a group of uneven cases, against the FP64 oracle.

From one shared state (rounded to complex64), the library and the oracle run
the same iteration (same order, same batches): every batch's update, the
complex constraint inside its window, the K-mode orthogonalisation at the end
of the iteration and the data error E_t.  Compared: the object on the union of
the scan boxes (relative L2 and worst element against the peak), the probe mode
by mode (the modes' powers are distinct, so the orthogonalised modes are
defined without ambiguity), the modes' powers (= the Gram eigenvalues after
orthogonalisation), sum_k |P_k|^2 per pixel, and E_t.

Bar: relative L2 <= 1e-5 (FP32 exit waves and updates); worst element <= 1e-4
of the peak (FP32 rounding of ~20 transform stages on one element, ~1e-6, with
margin for the dim pixels whose relative error the division by the blurred
amplitude amplifies); eigenvalues and E_t within 1e-5 relative.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as ora
from parity_util import inf_rel, params_pair, probe_metrics, rel_l2, union_of_boxes

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_INF = 1e-4


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _iterations_from_shared_state(s, cp, op, orders, roi):
    import paper_2406_06640_amd as P
    o32 = s["obj0"].astype(np.complex64)
    p32 = s["probe0"].astype(np.complex64)
    sq = ora.measured_amplitude(s["intensities"], op)
    out = []
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as rec:
        st = ora.State(O=o32.astype(np.complex128), P=p32.astype(np.complex128))
        for it in range(len(orders)):
            o_r, p_r = st.O.astype(np.complex64), st.P.astype(np.complex64)
            rec.set_state(o_r, p_r, it)
            st = ora.State(O=o_r.astype(np.complex128), P=p_r.astype(np.complex128), t=it)
            e_g = rec.iterate(1, orders[it:it + 1])
            st, e_o = ora.iterate(st, None, s["positions"], op, 1, orders=orders[it:it + 1], sqrt_I=sq)
            og, pg = rec.object(), rec.probe()
            r = dict(O=rel_l2(og[roi], st.O[roi]), O_inf=inf_rel(og[roi], st.O[roi]),
                     O_outside_untouched=bool(np.array_equal(og[~roi], o_r[~roi])),
                     P=rel_l2(pg, st.P), P_inf=inf_rel(pg, st.P), err=abs(float(e_g[0]) - e_o[0]) / abs(e_o[0]))
            r.update(probe_metrics(pg, st.P))
            print(it + 1, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
            out.append(r)
    return out


def _check(res):
    for r in res:
        assert r["O_outside_untouched"], r
        for key in ("O", "P", "sum_p2", "eig", "err"):
            assert r[key] <= TOL, (key, r)
        for key in ("O_inf", "P_inf", "sum_p2_inf"):
            assert r[key] <= TOL_INF, (key, r)


@pytest.mark.parametrize("cfg,n_pos,n_iter", [("far256_k4", 96, 2), ("near512_k8", 24, 1)])
def test_full_size_iterations(cfg, n_pos, n_iter):
    """256^2 frames, K = 4, B = 32 (3 batches; 5-wavelength data) and 512^2 near-field
    frames, K = 8, B = 8 (3 batches): constraint window on, orthogonalisation on."""
    import datagen
    spec = datagen.CONFIGS[cfg]
    s = datagen.make_scan(spec, spec["seed"], n_pos=n_pos, probe_known=True)
    B = spec["batch"]
    cp, op = params_pair(s, batch=B, cc_start=1, cc_end=10, orthogonalize=1)
    _announce(f"full-size iterations {cfg} n={cp.n} K={cp.n_modes} B={B} positions={n_pos}")
    orders = np.stack([ora.permutation(3, t, n_pos) for t in range(1, n_iter + 1)]).astype(np.int32)
    roi = union_of_boxes(s["positions"], s["n"], s["obj0"].shape)
    _check(_iterations_from_shared_state(s, cp, op, orders, roi))


def test_group_matches_oracle_per_case():
    """A group of three uneven cases (N = 64 / 128 / 192, K = 1 / 3 / 5, different
    batch sizes and position counts) for one iteration in its own generated orders,
    each case against the oracle's iteration in the same order."""
    import paper_2406_06640_amd as P
    from parity_util import make_case
    specs = [(dict(n=64, k=1, obj=(144, 144), n_side=5, step=16, radius=16, seed=61), dict(batch=7, seed=11)),
             (dict(n=128, k=3, obj=(224, 224), n_side=4, step=24, radius=32, seed=62),
              dict(batch=5, seed=12, cc_start=1, cc_end=3)),
             (dict(n=192, k=5, obj=(288, 288), n_side=3, step=40, radius=48, seed=63), dict(batch=4, seed=13))]
    _announce("group of 3 (N 64/128/192, K 1/3/5) vs oracle")
    made = []
    for ckw, pkw in specs:
        s = make_case(**ckw)
        s["probe0"] = s["probe_true"]  # distinct mode powers
        cp, op = params_pair(s, **pkw)
        made.append((s, cp, op))
    recs = []
    try:
        for s, cp, _ in made:
            recs.append(P.Reconstruction(cp, s["intensities"], s["positions"], s["probe0"].astype(np.complex64),
                                         s["obj0"].astype(np.complex64)))
        with P.Group(recs) as g:
            errs = g.iterate(1)
        for i, ((s, cp, op), r) in enumerate(zip(made, recs)):
            st = ora.State(O=s["obj0"].astype(np.complex64).astype(np.complex128),
                           P=s["probe0"].astype(np.complex64).astype(np.complex128))
            st, e_o = ora.iterate(st, s["intensities"], s["positions"], op, 1)
            roi = union_of_boxes(s["positions"], s["n"], s["obj0"].shape)
            og, pg = r.object(), r.probe()
            res = dict(O=rel_l2(og[roi], st.O[roi]), O_inf=inf_rel(og[roi], st.O[roi]), O_outside_untouched=True,
                       P=rel_l2(pg, st.P), P_inf=inf_rel(pg, st.P),
                       err=abs(float(errs[i][0]) - e_o[0]) / abs(e_o[0]))
            res.update(probe_metrics(pg, st.P))
            print(f"case {i} n={cp.n} K={cp.n_modes}",
                  {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in res.items()}, flush=True)
            _check([res])
    finally:
        for r in recs:
            r.close()
