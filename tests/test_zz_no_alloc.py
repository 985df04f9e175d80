"""ptycho_iterate_static (the entry point that allocates nothing: its per-call
buffers live in the library's static device scratch) against ptycho_iterate on
identical contexts, through the C ABI: two calls in a row, the second on a
smaller reconstruction (the scratch then holds the first call's contents), and
the size limit."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as ora
from parity_util import make_case, params_pair, state32

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _pair(s, cp, n_iter, order):
    import paper_2406_06640_amd as P
    o32, p32 = state32(s)
    out = []
    for static in (False, True):
        with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
            fn = P.ptycho_iterate_static if static else P.ptycho_iterate
            e = fn(r.ctx, n_iter, order)
            out.append((r.object(), r.probe(), e, r.iteration))
    return out


def test_static_entry_matches_iterate_twice_then_smaller():
    # first call: 64^2 frames, K = 3, 36 positions in batches of 5 (a ragged last batch),
    # constraint window and orthogonalisation on, generated order; second call: a
    # smaller reconstruction (32^2, K = 1, 16 positions, batch 2) with an explicit order
    big = make_case(n=64, k=3, obj=(128, 128), n_side=6, step=12, radius=16, seed=71)
    cp_b, _ = params_pair(big, batch=5, cc_start=1, cc_end=2, seed=4)
    small = make_case(n=32, k=1, obj=(64, 64), n_side=4, step=8, seed=72)
    cp_s, _ = params_pair(small, batch=2)
    orders = np.stack([ora.permutation(9, t, 16) for t in (1, 2)]).astype(np.int32)
    for name, s, cp, n_iter, order in (("big", big, cp_b, 3, None), ("small", small, cp_s, 2, orders)):
        _announce(f"static vs iterate: {name} n={cp.n} K={cp.n_modes} B={cp.batch} iterations={n_iter}")
        (o_a, p_a, e_a, t_a), (o_b, p_b, e_b, t_b) = _pair(s, cp, n_iter, order)
        np.testing.assert_array_equal(o_b, o_a)
        np.testing.assert_array_equal(p_b, p_a)
        np.testing.assert_array_equal(e_b, e_a)
        assert t_a == t_b == n_iter


def test_static_entry_continues_a_context_and_rejects_oversize():
    import paper_2406_06640_amd as P
    s = make_case(n=32, k=2, obj=(80, 80), n_side=5, step=8, seed=73)
    cp, _ = params_pair(s, batch=4, probe_update_start=2)
    _announce("static entry mixed with iterate on one context")
    o32, p32 = state32(s)
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        e1 = P.ptycho_iterate(r.ctx, 2)
        e2 = P.ptycho_iterate_static(r.ctx, 1)
        e3 = P.ptycho_iterate(r.ctx, 1)
        mixed = (r.object(), r.probe(), np.concatenate([e1, e2, e3]))
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        e = P.ptycho_iterate(r.ctx, 4)
        np.testing.assert_array_equal(mixed[0], r.object())
        np.testing.assert_array_equal(mixed[1], r.probe())
        np.testing.assert_array_equal(mixed[2], e)
    # 256^2 frames, K = 4, batch 32: ~100 MB of work buffers, over the 64 MiB limit
    big = make_case(n=256, k=4, obj=(320, 320), n_side=2, step=32, radius=64, seed=74)
    cpb, _ = params_pair(big, batch=32)
    _announce("static entry size limit")
    o32, p32 = state32(big)
    with P.Reconstruction(cpb, big["intensities"], big["positions"], p32, o32) as r:
        with pytest.raises(P.PtychoError) as ei:
            P.ptycho_iterate_static(r.ctx, 1)
        assert ei.value.status == P.PTYCHO_E_SHAPE
        assert "scratch" in str(ei.value)
        assert r.iteration == 0
