"""Pins for the ePIE loop of Fig. 1 as the oracle implements it.

The references here are written independently in the test: textbook ePIE and
rPIE single-position steps (refs. [24], [25] of the paper) using numpy's
unnormalised FFT, compared with the oracle's batched step in the cases where
the batched rule must reduce to them.
"""

import numpy as np
import pytest

import oracle as ora


def _scan(rng, obj=40, n=16, k=1):
    O = (0.8 + 0.2 * rng.random((obj, obj))) * np.exp(1j * (rng.random((obj, obj)) - 0.5))
    y, x = np.mgrid[0:n, 0:n]
    ap = ((x - n / 2) ** 2 + (y - n / 2) ** 2 <= (n / 3) ** 2).astype(complex)
    P = np.stack([ap * np.exp(1j * 0.3 * (m + 1) * x / n) * (0.7 ** m) for m in range(k)])
    pos = np.array([(2, 3), (10, 5), (7, 20), (20, 18), (24, 2), (3, 24)], dtype=np.int32)
    meas = rng.random((len(pos), n, n)) * 4.0
    return O, P, pos, meas


def _textbook_step(O, P, pos, meas_fft_order, alpha, beta, gamma_o=1.0, gamma_p=1.0, probe=True):
    """Single-position ePIE / rPIE, fully coherent, written from the published
    update rules with numpy's unnormalised FFT."""
    n = P.shape[-1]
    r, c = pos
    o = O[r:r + n, c:c + n].copy()
    p = P[0]
    psi = o * p
    Psi = np.fft.fft2(psi) / n
    Psi_new = meas_fft_order * np.exp(1j * np.angle(Psi))
    dpsi = np.fft.ifft2(Psi_new * n) - psi
    p2 = np.abs(p) ** 2
    o2 = np.abs(o) ** 2
    O2 = O.copy()
    O2[r:r + n, c:c + n] = o + alpha * np.conj(p) * dpsi / ((1 - gamma_o) * p2 + gamma_o * p2.max())
    P2 = P.copy()
    if probe:
        P2[0] = p + beta * np.conj(o) * dpsi / ((1 - gamma_p) * o2 + gamma_p * o2.max())
    return O2, P2


@pytest.mark.parametrize("gammas", [(1.0, 1.0), (0.3, 0.6)])
def test_batch_of_one_is_textbook_epie_or_rpie(gammas, rng):
    O, P, pos, meas = _scan(rng)
    n = P.shape[-1]
    params = ora.Params(n=n, sigma1=0.0, sigma2=0.0, eps=0.0, batch=1, obj_step=0.9, probe_step=0.7,
                        gamma_obj=gammas[0], gamma_probe=gammas[1])
    sq = np.fft.ifftshift(meas, axes=(-2, -1))
    Oa, Pa = O.copy(), P.copy()
    Ob, Pb = O.copy(), P.copy()
    for i in [3, 0, 5, 1]:
        Oa, Pa, _, _ = ora.batch_step(Oa, Pa, sq, pos, [i], 1, params)
        Ob, Pb = _textbook_step(Ob, Pb, pos[i], sq[i], 0.9, 0.7, *gammas)
    np.testing.assert_allclose(Oa, Ob, atol=1e-12)
    np.testing.assert_allclose(Pa, Pb, atol=1e-12)


def test_probe_update_start_freezes_probe(rng):
    O, P, pos, meas = _scan(rng)
    params = ora.Params(n=16, sigma1=0.0, sigma2=0.0, probe_update_start=3)
    sq = np.fft.ifftshift(meas, axes=(-2, -1))
    _, P2, _, _ = ora.batch_step(O, P, sq, pos, [0], 2, params)
    np.testing.assert_array_equal(P2, P)
    _, P3, _, _ = ora.batch_step(O, P, sq, pos, [0], 3, params)
    assert np.abs(P3 - P).max() > 0


def test_disjoint_batch_equals_sequential_object_steps(rng):
    """Two non-overlapping boxes with the probe frozen: the batched object
    update equals two sequential textbook steps (max W is the same for both)."""
    O, P, pos, meas = _scan(rng)
    sq = np.fft.ifftshift(meas, axes=(-2, -1))
    params = ora.Params(n=16, sigma1=0.0, sigma2=0.0, eps=0.0, batch=2, probe_update_start=99)
    i, j = 0, 3  # boxes at (2,3) and (20,18) do not overlap for n = 16
    Oa, _, _, _ = ora.batch_step(O, P, sq, pos, [i, j], 1, params)
    Ob, _ = _textbook_step(O, P, pos[i], sq[i], 1.0, 1.0, probe=False)
    Ob, _ = _textbook_step(Ob, P, pos[j], sq[j], 1.0, 1.0, probe=False)
    np.testing.assert_allclose(Oa, Ob, atol=1e-12)


def test_consistent_state_is_fixed_point(rng):
    """Data generated from (O, P) with sigma = 0: every step leaves O and P unchanged."""
    O, P, pos, _ = _scan(rng, k=2)
    n = P.shape[-1]
    params = ora.Params(n=n, n_modes=2, sigma1=0.0, sigma2=0.0, eps=0.0, batch=3)
    amp = np.stack([np.sqrt(np.sum(np.abs(np.fft.fft2(O[r:r + n, c:c + n] * P, norm="ortho")) ** 2,
                                   axis=0)) for (r, c) in pos])
    O2, P2, err, _ = ora.batch_step(O, P, amp, pos, [0, 2, 4], 1, params)
    np.testing.assert_allclose(O2, O, atol=1e-12)
    np.testing.assert_allclose(P2, P, atol=1e-12)
    assert err < 1e-20


def test_batched_accumulators_against_per_position_sums(rng):
    """N_O, W, N_P, V of an overlapping batch equal the per-position terms
    summed at the box offsets (captured exit waves give dpsi)."""
    O, P, pos, meas = _scan(rng, k=2)
    n = 16
    sq = np.fft.ifftshift(meas, axes=(-2, -1))
    params = ora.Params(n=n, n_modes=2, sigma1=1.0, sigma2=1.0, batch=3)
    batch = [1, 0, 2]
    _, _, _, cap = ora.batch_step(O, P, sq, pos, batch, 1, params, capture=True)
    n_o = np.zeros_like(O)
    w = np.zeros(O.shape)
    for b, i in enumerate(batch):
        r, c = pos[i]
        d = cap["psi_new"][b] - cap["psi"][b]
        n_o[r:r + n, c:c + n] += np.sum(np.conj(P) * d, axis=0)
        w[r:r + n, c:c + n] += np.sum(np.abs(P) ** 2, axis=0)
        np.testing.assert_allclose(cap["psi"][b], O[r:r + n, c:c + n] * P, atol=1e-14)
    np.testing.assert_allclose(cap["n_o"], n_o, atol=1e-12)
    np.testing.assert_allclose(cap["w"], w, atol=1e-12)


def test_permutation_is_deterministic_permutation():
    a = ora.permutation(7, 1, 100)
    assert sorted(a.tolist()) == list(range(100))
    np.testing.assert_array_equal(a, ora.permutation(7, 1, 100))
    assert not np.array_equal(a, ora.permutation(7, 2, 100))
    assert ora.permutation(7, 1, 1).tolist() == [0]
    assert ora.permutation(7, 1, 0).tolist() == []


def test_iteration_error_decreases_noise_free(rng):
    """Data error E_t of a noise-free, fully coherent scan falls as ePIE iterates."""
    import datagen
    spec = dict(datagen.CONFIGS["far64"])
    spec.update(obj=(48, 48), n=16, n_side=4, step=6, radius=5, jitter=0, sigma_data=0.0)
    s = datagen.make_scan(spec, 5, noise=False, probe_known=True)
    params = ora.Params(n=16, sigma1=0.0, sigma2=0.0, probe_update_start=1000, batch=1)
    st = ora.State(O=s["obj0"], P=s["probe0"])
    st, errs = ora.iterate(st, s["intensities"], s["positions"], params, 30)
    assert errs[-1] < 0.2 * errs[0]
    assert errs[-1] < errs[10]
