"""Pins of the FP64 pc-DM oracle (oracle/pcdm.py) against what the difference
map's definition fixes: the overlap projection is the regularised
least-squares solution (checked by brute force on a small stacked system),
consistent data make the exact state a fixed point, with one scan position and
no regularisation the step reduces to the textbook Fourier-modulus projection
(error reduction), and on noise-free data the iteration converges to the truth."""

import numpy as np

import oracle as ora
from oracle import pcdm


def _tiny(rng, n=6, obj=(12, 11), pos=((0, 0), (3, 2), (5, 5), (2, 4)), k=2):
    O = rng.standard_normal(obj) + 1j * rng.standard_normal(obj)
    P = rng.standard_normal((k, n, n)) + 1j * rng.standard_normal((k, n, n))
    positions = np.array(pos, dtype=np.int64)
    psi = rng.standard_normal((len(positions), k, n, n)) + 1j * rng.standard_normal((len(positions), k, n, n))
    return O, P, positions, psi


def test_object_projection_is_regularised_least_squares(rng):
    O, P, positions, psi = _tiny(rng)
    n, delta = P.shape[-1], 0.05
    got, mask = pcdm.project_object(psi, O, P, positions, delta)
    # brute force: unknowns are the object pixels; one row per (position, mode, box pixel)
    # with coefficient P_k, plus sqrt(reg) rows pulling every pixel of the boxes to O
    h, w = O.shape
    rows, rhs = [], []
    for i, (r, c) in enumerate(positions):
        for k in range(P.shape[0]):
            for y in range(n):
                for x in range(n):
                    a = np.zeros(h * w, complex)
                    a[(r + y) * w + (c + x)] = P[k, y, x]
                    rows.append(a)
                    rhs.append(psi[i, k, y, x])
    wmax = 0.0
    wmap = np.zeros((h, w))
    for (r, c) in positions:
        wmap[r:r + n, c:c + n] += np.sum(np.abs(P) ** 2, axis=0)
    wmax = wmap.max()
    idx = np.flatnonzero(mask.ravel())
    for j in idx:
        a = np.zeros(h * w, complex)
        a[j] = np.sqrt(delta * wmax)
        rows.append(a)
        rhs.append(np.sqrt(delta * wmax) * O.ravel()[j])
    A = np.array(rows)[:, idx]
    sol, *_ = np.linalg.lstsq(A, np.array(rhs), rcond=None)
    np.testing.assert_allclose(got.ravel()[idx], sol, atol=1e-10)
    np.testing.assert_array_equal(got[~mask], O[~mask])


def test_probe_projection_is_regularised_least_squares(rng):
    O, P, positions, psi = _tiny(rng, k=3)
    n, delta = P.shape[-1], 0.02
    got = pcdm.project_probe(psi, O, P, positions, delta)
    v = np.zeros((n, n))
    for (r, c) in positions:
        v += np.abs(O[r:r + n, c:c + n]) ** 2
    reg = delta * v.max()
    for k in range(P.shape[0]):
        for y in range(n):
            for x in range(n):
                # one unknown: rows o_n(y, x) (one per position) and the pull sqrt(reg)
                a = [O[r + y, c + x] for (r, c) in positions] + [np.sqrt(reg)]
                b = [psi[i, k, y, x] for i in range(len(positions))] + [np.sqrt(reg) * P[k, y, x]]
                sol, *_ = np.linalg.lstsq(np.array(a)[:, None], np.array(b), rcond=None)
                assert abs(got[k, y, x] - sol[0]) < 1e-11


def _consistent(rng, n=16, k=2, sigma=0.0, blur_domain=ora.BLUR_AMPLITUDE):
    O = np.exp(0.3j * rng.standard_normal((40, 40))) * (0.8 + 0.2 * rng.random((40, 40)))
    y, x = np.mgrid[0:n, 0:n] - n / 2
    base = (x * x + y * y <= (n / 3) ** 2) * np.exp(0.1j * (x * x + y * y))
    P = np.stack([base * (1.0 if j == 0 else 0.3 * (x / n + 0.1j * y / n) ** j) for j in range(k)])
    positions = np.array([(r, c) for r in (0, 8, 16, 24) for c in (0, 9, 17, 24)])
    params = ora.Params(n=n, n_modes=k, sigma1=sigma, sigma2=sigma, blur_domain=blur_domain, batch=1)
    g = ora.gaussian_kernel(sigma, sigma, params.kernel_size)
    z = pcdm.exit_waves(O, P, positions)
    inten = np.zeros((len(positions), n, n))
    for i in range(len(positions)):
        i_mod = np.sum(np.abs(ora.fft2u(z[i])) ** 2, axis=0)
        inten[i] = ora.blur_periodic(i_mod, g) if sigma > 0 else i_mod
    sq = np.sqrt(inten)  # FFT order already
    return O, P, positions, params, sq


def test_consistent_data_is_a_fixed_point(rng):
    # exact state, data consistent with it (no blur; and the intensity blur of Eq. 2 applied
    # to both the data and the model): one iteration changes nothing
    for sigma, dom in ((0.0, ora.BLUR_AMPLITUDE), (1.2, ora.BLUR_INTENSITY)):
        O, P, positions, params, sq = _consistent(rng, sigma=sigma, blur_domain=dom)
        params.eps = 0.0
        st = pcdm.initial_state(O, P, positions)
        new, err = pcdm.dm_iteration(st, sq, positions, params, delta=1e-3)
        np.testing.assert_allclose(new.O, O, atol=1e-10)
        np.testing.assert_allclose(new.P, P, atol=1e-10)
        np.testing.assert_allclose(new.psi, st.psi, atol=1e-10)
        assert err < 1e-18 * np.sum(sq ** 2) + 1e-20


def test_single_position_reduces_to_fourier_projection(rng):
    # one box, no regularisation, a probe without zeros, probe frozen: the overlap
    # projection returns z = psi, so the step is psi <- P_F(psi), the modulus projection
    n = 8
    O = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    P = (1.0 + rng.random((1, n, n))) * np.exp(1j * rng.standard_normal((1, n, n)))
    psi = rng.standard_normal((1, 1, n, n)) + 1j * rng.standard_normal((1, 1, n, n))
    sq = rng.random((1, n, n)) + 0.5
    params = ora.Params(n=n, sigma1=0.0, sigma2=0.0, kernel_size=1, eps=0.0, probe_update_start=10)
    st = pcdm.DMState(O=O, P=P, psi=psi, t=0)
    new, _ = pcdm.dm_iteration(st, sq, np.array([(0, 0)]), params, delta=1e-14)
    Psi = np.fft.fft2(psi[0, 0], norm="ortho")
    expect = np.fft.ifft2(sq[0] * Psi / np.abs(Psi), norm="ortho")
    np.testing.assert_allclose(new.psi[0, 0], expect, atol=1e-9)


def test_noise_free_convergence_with_known_probe():
    import datagen
    spec = dict(datagen.CONFIGS["far64"])
    spec.update(obj=(48, 48), n=16, n_side=4, step=6, radius=5, jitter=0, sigma_data=0.0)
    s = datagen.make_scan(spec, 5, noise=False, probe_known=True)
    params = ora.Params(n=16, sigma1=0.0, sigma2=0.0, kernel_size=1, probe_update_start=1000)
    st = pcdm.initial_state(s["obj0"], s["probe0"], s["positions"])
    roi = ora.illumination_roi(s["positions"], s["probe_true"], s["obj_true"].shape)
    e0 = ora.nmse(st.O, s["obj_true"], roi)
    st, errs = pcdm.dm_iterate(st, s["intensities"], s["positions"], params, 60)
    e1 = ora.nmse(st.O, s["obj_true"], roi)
    # the object converges to the truth (the data error of the reflected estimate 2z - psi
    # that E_t measures levels off at the map's fixed point, where psi differs from z)
    assert e1 < 1e-3 and e1 < 0.01 * e0
    assert errs[-1] < 0.6 * errs[0]
