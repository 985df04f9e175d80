"""GPU checks of the batched execution paths: groups of independent
reconstructions of uneven size advanced together, iteration replay from a
captured HIP graph, and the column-tile autotuner.  Each must reproduce the
plain single-context run bitwise (the object, the probe and the data error)."""

from __future__ import annotations

import numpy as np
import pytest

from parity_util import make_case, params_pair, state32

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


CASES = [
    # (make_case kwargs, params kwargs)
    (dict(n=32, k=2, obj=(80, 80), n_side=5, step=8, seed=31), dict(batch=4, cc_start=1, cc_end=2, seed=5)),
    (dict(n=64, k=1, obj=(144, 144), n_side=6, step=12, radius=16, seed=32), dict(batch=7, seed=6)),
    (dict(n=32, k=3, obj=(72, 72), n_side=4, step=8, seed=33), dict(batch=3, probe_update_start=2, seed=7)),
    (dict(n=48, k=2, geometry=1, obj=(96, 96), n_side=3, step=12, radius=12, seed=34),
     dict(batch=2, sigma1=1.5, sigma2=1.5, seed=8)),
    (dict(n=64, k=4, obj=(128, 128), n_side=3, step=16, radius=16, seed=35), dict(batch=9, cc_start=2, cc_end=3,
                                                                                  seed=9)),
    (dict(n=64, k=2, geometry=1, obj=(128, 128), n_side=3, step=16, radius=16, seed=36), dict(batch=5, seed=10)),
]


def _make(idx):
    ckw, pkw = CASES[idx]
    s = make_case(**ckw)
    cp, _ = params_pair(s, **pkw)
    return s, cp


def _run_single(s, cp, n_iter, graph=False, chunks=None):
    import paper_2406_06640_amd as P
    o32, p32 = state32(s)
    errs = []
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        if graph:
            r.set_graph(True)
        for n in (chunks or [n_iter]):
            errs.append(r.iterate(n))
            # eager host work and synchronisation between replays
            _ = r.object()
        return r.object(), r.probe(), np.concatenate(errs)


def test_group_matches_single_runs():
    import paper_2406_06640_amd as P
    _announce("group of 5 uneven cases vs single runs")
    made = [_make(i) for i in range(len(CASES))]
    singles = [_run_single(s, cp, 3) for s, cp in made]
    recs = []
    try:
        for s, cp in made:
            o32, p32 = state32(s)
            recs.append(P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32))
        with P.Group(recs) as g:
            errs = g.iterate(2)
            errs = np.concatenate([errs, g.iterate(1)], axis=1)
        for i, r in enumerate(recs):
            o, p, e = singles[i]
            np.testing.assert_array_equal(r.object(), o, err_msg=f"case {i} object")
            np.testing.assert_array_equal(r.probe(), p, err_msg=f"case {i} probe")
            np.testing.assert_array_equal(errs[i], e, err_msg=f"case {i} error")
            assert r.iteration == 3
    finally:
        for r in recs:
            r.close()


def test_group_graph_replay_matches_eager_group():
    import paper_2406_06640_amd as P
    _announce("group of 5 uneven cases, graph replay vs eager")
    made = [_make(i) for i in range(len(CASES))]
    results = []
    for graph in (False, True):
        recs = []
        try:
            for s, cp in made:
                o32, p32 = state32(s)
                recs.append(P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32))
            with P.Group(recs) as g:
                g.set_graph(graph)
                errs = [g.iterate(2)]
                _ = recs[0].object()  # eager host work between replays
                errs.append(g.iterate(1))
                errs.append(g.iterate(2))
            results.append(([r.object() for r in recs], [r.probe() for r in recs], np.concatenate(errs, axis=1)))
        finally:
            for r in recs:
                r.close()
    (oe, pe, ee), (og, pg, eg) = results
    for i in range(len(CASES)):
        np.testing.assert_array_equal(og[i], oe[i], err_msg=f"case {i} object")
        np.testing.assert_array_equal(pg[i], pe[i], err_msg=f"case {i} probe")
    np.testing.assert_array_equal(eg, ee)


@pytest.mark.parametrize("case", [0, 3, 4])
def test_graph_replay_matches_eager(case):
    s, cp = _make(case)
    _announce(f"graph replay case {case}")
    o_e, p_e, e_e = _run_single(s, cp, 5)
    o_g, p_g, e_g = _run_single(s, cp, 5, graph=True, chunks=[2, 1, 2])
    np.testing.assert_array_equal(o_g, o_e)
    np.testing.assert_array_equal(p_g, p_e)
    np.testing.assert_array_equal(e_g, e_e)


@pytest.mark.parametrize("case", [1, 4, 5])
def test_every_launch_variant_gives_the_same_result(case):
    """Column widths and mode-parallel passes change only the launch shape."""
    import paper_2406_06640_amd as P
    s, cp = _make(case)
    _announce(f"all launch variants, case {case}")
    o32, p32 = state32(s)
    ref = None
    ran = []
    for v in range(P.ptycho_variant_count()):
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            try:
                r.set_variant(v)
            except P.PtychoError:
                continue
            r.iterate(2)
            got = (r.object(), r.probe())
        ran.append(v)
        if ref is None:
            ref = got
        else:
            np.testing.assert_array_equal(got[0], ref[0], err_msg=f"variant {v} object")
            np.testing.assert_array_equal(got[1], ref[1], err_msg=f"variant {v} probe")
    print(f"variants run: {ran}", flush=True)
    assert len(ran) >= 12


@pytest.mark.parametrize("n,k", [(128, 3), (192, 2), (256, 1), (256, 4)])
def test_launch_variants_agree_for_larger_frames(n, k):
    """Every launch variant of the larger frame sizes, one batch step, bitwise."""
    import paper_2406_06640_amd as P
    s = make_case(n=n, k=k, obj=(n + 64, n + 64), n_side=3, step=24, radius=n // 4, seed=40 + n + k)
    cp, _ = params_pair(s, batch=5, cc_start=1, cc_end=2, seed=3)
    _announce(f"launch variants n={n} K={k}")
    o32, p32 = state32(s)
    ref, ran = None, []
    for v in range(P.ptycho_variant_count()):
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            try:
                r.set_variant(v)
            except P.PtychoError:
                continue
            r.iterate(1)
            got = (r.object(), r.probe())
        ran.append(v)
        if ref is None:
            ref = got
        else:
            np.testing.assert_array_equal(got[0], ref[0], err_msg=f"variant {v} object")
            np.testing.assert_array_equal(got[1], ref[1], err_msg=f"variant {v} probe")
    print(f"variants run: {ran}", flush=True)
    assert len(ran) >= 12


def test_autotune_choice_keeps_results():
    """Every column-tile variant gives the same object and probe."""
    import paper_2406_06640_amd as P
    s, cp = _make(4)
    _announce("autotune n=64 K=4")
    ref = _run_single(s, cp, 2)
    o32, p32 = state32(s)
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        v = r.autotune(trials=2, force=True)
        assert 0 <= v < P.ptycho_variant_count()
        # the state is restored by the tuner
        np.testing.assert_array_equal(r.object(), o32)
        np.testing.assert_array_equal(r.probe(), p32)
        r.iterate(2)
        np.testing.assert_array_equal(r.object(), ref[0])
        np.testing.assert_array_equal(r.probe(), ref[1])
