"""GPU parity of the pc-DM engine (the difference map with the blurred modulus
projection and the complex constraint, Sec. 4.5) against the FP64 oracle
(oracle/pcdm.py), through the C ABI.

From one shared state (object, probe and the exit waves of every position,
rounded to complex64) both run the same iteration; compared: the object on the
union of the boxes, the probe, every exit wave and the data error E_t, within
the spec bar of 1e-5 relative L2 (FP32 transforms and updates) and a
worst element within 1e-4 of the peak.  Also: the Fourier step's batching does
not change the result (bitwise), runs are bitwise reproducible, exit waves
round-trip through the ABI, and the ePIE-only entry points refuse a DM context.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as ora
from oracle import pcdm
from parity_util import inf_rel, make_case, params_pair, rel_l2, union_of_boxes

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_INF = 1e-4
DELTA = 1e-3


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _dm_params(s, **kw):
    import paper_2406_06640_amd as P
    cp, op = params_pair(s, **kw)
    cp.engine = P.PTYCHO_ENGINE_DM
    cp.dm_reg = DELTA
    return cp, op


def _perturbed_state(s, rng):
    """A state away from the start (so every term of the update matters): the initial
    object and probe with small random perturbations, exit waves P o_n plus noise."""
    o = s["obj0"] * (1.0 + 0.05 * (rng.standard_normal(s["obj0"].shape) + 1j * rng.standard_normal(s["obj0"].shape)))
    p = s["probe0"] * (1.0 + 0.05 * rng.standard_normal(s["probe0"].shape))
    o, p = o.astype(np.complex64), p.astype(np.complex64)
    psi = pcdm.exit_waves(o.astype(np.complex128), p.astype(np.complex128), s["positions"])
    scale = np.sqrt(np.mean(np.abs(psi) ** 2))
    psi = psi + 0.1 * scale * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    return o, p, psi.astype(np.complex64)


def _iterate_shared(s, cp, op, n_iter, seed=1):
    import paper_2406_06640_amd as P
    rng = np.random.default_rng(seed)
    o, p, psi = _perturbed_state(s, rng)
    sq = ora.measured_amplitude(s["intensities"], op)
    g = ora.gaussian_kernel(op.sigma1, op.sigma2, op.kernel_size)
    denom = float(np.sum(sq ** 2))
    roi = union_of_boxes(s["positions"], s["n"], s["obj0"].shape)
    out = []
    with P.Reconstruction(cp, s["intensities"], s["positions"], p, o) as r:
        st = pcdm.DMState(O=o.astype(np.complex128), P=p.astype(np.complex128), psi=psi.astype(np.complex128), t=0)
        for it in range(n_iter):
            o_r, p_r, s_r = st.O.astype(np.complex64), st.P.astype(np.complex64), st.psi.astype(np.complex64)
            r.set_state(o_r, p_r, it)
            r.set_exit_waves(s_r)
            st = pcdm.DMState(O=o_r.astype(np.complex128), P=p_r.astype(np.complex128),
                              psi=s_r.astype(np.complex128), t=it)
            e_g = r.iterate(1)
            st, e_o = pcdm.dm_iteration(st, sq, s["positions"], op, DELTA, g)
            og, pg, sg = r.object(), r.probe(), r.exit_waves()
            res = dict(O=rel_l2(og[roi], st.O[roi]), O_inf=inf_rel(og[roi], st.O[roi]), P=rel_l2(pg, st.P),
                       P_inf=inf_rel(pg, st.P), psi=rel_l2(sg, st.psi), psi_inf=inf_rel(sg, st.psi),
                       err=abs(float(e_g[0]) - e_o / denom) / (e_o / denom),
                       outside=bool(np.array_equal(og[~roi], o_r[~roi])))
            print(it + 1, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in res.items()}, flush=True)
            out.append(res)
    return out


CASES = {
    # name: (make_case kwargs, params kwargs, iterations)
    "far_n64_k1_window": (dict(n=64, obj=(128, 128), n_side=6, step=12, radius=16, seed=81),
                          dict(batch=8, cc_start=1, cc_end=3, alpha1=0.8, alpha2=0.1), 2),
    "far_n32_k2_intensity": (dict(n=32, k=2, obj=(80, 80), n_side=5, step=8, seed=82),
                             dict(batch=5, blur_domain=1, sigma1=0.8, sigma2=1.2, kernel_size=7), 2),
    "near_n64_k2": (dict(n=64, k=2, geometry=1, obj=(128, 128), n_side=4, step=16, radius=16, seed=83),
                    dict(batch=4, sigma1=1.5, sigma2=1.5), 1),
    "probe_frozen_radix3": (dict(n=48, k=1, obj=(96, 96), n_side=4, step=12, radius=12, seed=84),
                            dict(batch=16, probe_update_start=5), 1),
    "far_n256_k4_full_frame": (dict(n=256, k=4, obj=(448, 448), n_side=5, step=40, radius=64, seed=85),
                               dict(batch=8, sigma1=2.0, sigma2=2.0, cc_start=1, cc_end=1), 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_dm_iteration_parity(name):
    ckw, pkw, n_iter = CASES[name]
    s = make_case(**ckw)
    cp, op = _dm_params(s, **pkw)
    _announce(f"pc-DM {name} n={cp.n} K={cp.n_modes} positions={len(s['positions'])} batch={cp.batch}")
    for r in _iterate_shared(s, cp, op, n_iter):
        assert r["outside"], r
        for key in ("O", "P", "psi", "err"):
            assert r[key] <= TOL, (key, r)
        for key in ("O_inf", "P_inf", "psi_inf"):
            assert r[key] <= TOL_INF, (key, r)


def test_dm_batching_and_determinism():
    """The Fourier step's batch size only groups launches: batch 3 and batch 36 give bitwise
    the same iterations, and a second run repeats them bitwise."""
    import paper_2406_06640_amd as P
    s = make_case(n=32, k=2, obj=(96, 96), n_side=6, step=10, seed=86)
    _announce("pc-DM batch independence and determinism")
    runs = []
    for batch in (3, 36, 3):
        cp, _ = _dm_params(s, batch=batch, cc_start=2, cc_end=3)
        with P.Reconstruction(cp, s["intensities"], s["positions"], s["probe0"].astype(np.complex64),
                              s["obj0"].astype(np.complex64)) as r:
            e = r.iterate(4)
            runs.append((r.object(), r.probe(), r.exit_waves(), e))
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            np.testing.assert_array_equal(a, b)


def test_dm_state_round_trip_and_refusals():
    import paper_2406_06640_amd as P
    s = make_case(n=32, k=1, obj=(72, 72), n_side=4, step=8, seed=87)
    cp, _ = _dm_params(s, batch=4)
    _announce("pc-DM exit-wave round trip and refusals")
    o32, p32 = s["obj0"].astype(np.complex64), s["probe0"].astype(np.complex64)
    with P.Reconstruction(cp, s["intensities"], s["positions"], p32, o32) as r:
        # the state starts at P o_n
        expect = pcdm.exit_waves(o32.astype(np.complex128), p32.astype(np.complex128), s["positions"])
        assert rel_l2(r.exit_waves(), expect) < 1e-6
        r.iterate(2)
        psi2, o2, p2 = r.exit_waves(), r.object(), r.probe()
        e3 = r.iterate(1)
        o3 = r.object()
        # resume from the saved state: bitwise the same third iteration
        r.set_state(o2, p2, 2)
        r.set_exit_waves(psi2)
        np.testing.assert_array_equal(r.iterate(1), e3)
        np.testing.assert_array_equal(r.object(), o3)
        with pytest.raises(P.PtychoError):
            P.ptycho_iterate_static(r.ctx, 1)
        with pytest.raises(P.PtychoError):
            P.Group([r])
