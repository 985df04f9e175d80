"""Pins of the FP64 pc-LSQML oracle (oracle/pclsqml.py) against what least
squares and the method's definition fix: the step pair is the minimiser of the
linearised exit-wave misfit (checked by a library least-squares solve on the
stacked real system, undamped and damped), consistent data make the exact state
a fixed point, with one position and no regularisation the object step lands
the exit wave exactly on the Fourier-modulus projection, the object and probe
directions of one position give the closed-form steps 1 / (2 + lam), and on
noise-free data the iteration converges to the truth."""

import numpy as np
import pytest

import oracle as ora
from oracle import pclsqml


def _cplx(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _stacked(chi, dO_j, P, o_j, dP):
    """The misfit sum_k ||chi_k - a dO_j P_k - b o_j dP_k||^2 as a real least-squares
    system A [a, b] ~ c (real and imaginary parts of every pixel and mode as rows)."""
    col_a = (dO_j[None] * P).ravel()
    col_b = (o_j[None] * dP).ravel()
    A = np.stack([np.concatenate([col_a.real, col_a.imag]), np.concatenate([col_b.real, col_b.imag])], axis=1)
    c = np.concatenate([chi.ravel().real, chi.ravel().imag])
    return A, c


@pytest.mark.parametrize("k", [1, 3])
def test_step_pair_is_the_least_squares_minimiser(rng, k):
    n = 7
    chi, P, dP = _cplx(rng, k, n, n), _cplx(rng, k, n, n), _cplx(rng, k, n, n)
    dO_j, o_j = _cplx(rng, n, n), _cplx(rng, n, n)
    M, r = pclsqml.lsq_normal_equations(chi, dO_j, P, o_j, dP)
    a, b = pclsqml.lsq_steps(M, r, 0.0, True)
    A, c = _stacked(chi, dO_j, P, o_j, dP)
    sol, *_ = np.linalg.lstsq(A, c, rcond=None)
    np.testing.assert_allclose([a, b], sol, rtol=1e-10)
    # the misfit at the step is below that at any nearby pair and below ||chi||^2
    f = lambda x, y: np.sum((A @ np.array([x, y]) - c) ** 2)
    best = f(a, b)
    for da, db in ((1e-3, 0), (-1e-3, 0), (0, 1e-3), (0, -1e-3), (1e-3, 1e-3)):
        assert f(a + da, b + db) > best
    assert best <= np.sum(np.abs(chi) ** 2)


def test_damped_step_pair_is_the_damped_least_squares_minimiser(rng):
    n, k, lam = 6, 2, 0.35
    chi, P, dP = _cplx(rng, k, n, n), _cplx(rng, k, n, n), _cplx(rng, k, n, n)
    dO_j, o_j = _cplx(rng, n, n), _cplx(rng, n, n)
    M, r = pclsqml.lsq_normal_equations(chi, dO_j, P, o_j, dP)
    a, b = pclsqml.lsq_steps(M, r, lam, True)
    A, c = _stacked(chi, dO_j, P, o_j, dP)
    # minimise ||A x - c||^2 + lam (M11 a^2 + M22 b^2), with M11, M22 the squared column norms
    m11, m22 = np.sum(A[:, 0] ** 2), np.sum(A[:, 1] ** 2)
    A_aug = np.vstack([A, [np.sqrt(lam * m11), 0.0], [0.0, np.sqrt(lam * m22)]])
    c_aug = np.concatenate([c, [0.0, 0.0]])
    sol, *_ = np.linalg.lstsq(A_aug, c_aug, rcond=None)
    np.testing.assert_allclose([a, b], sol, rtol=1e-10)
    # without probe update only the object step is free
    a1, b1 = pclsqml.lsq_steps(M, r, lam, False)
    sol1, *_ = np.linalg.lstsq(np.vstack([A[:, :1], [[np.sqrt(lam * m11)]]]), c_aug[:-1], rcond=None)
    assert b1 == 0.0 and abs(a1 - sol1[0]) < 1e-10 * abs(sol1[0])


def _consistent(rng, n=16, k=2, sigma=0.0, blur_domain=ora.BLUR_AMPLITUDE):
    O = np.exp(0.3j * rng.standard_normal((40, 40))) * (0.8 + 0.2 * rng.random((40, 40)))
    y, x = np.mgrid[0:n, 0:n] - n / 2
    base = (x * x + y * y <= (n / 3) ** 2) * np.exp(0.1j * (x * x + y * y))
    P = np.stack([base * (1.0 if j == 0 else 0.3 * (x / n + 0.1j * y / n) ** j) for j in range(k)])
    positions = np.array([(r, c) for r in (0, 8, 16, 24) for c in (0, 9, 17, 24)])
    params = ora.Params(n=n, n_modes=k, sigma1=sigma, sigma2=sigma, blur_domain=blur_domain, batch=4,
                        gamma_obj=0.2, gamma_probe=0.2)
    g = ora.gaussian_kernel(sigma, sigma, params.kernel_size)
    sq = np.zeros((len(positions), n, n))
    for i, (r, c) in enumerate(positions):
        i_mod = np.sum(np.abs(ora.fft2u(O[r:r + n, c:c + n][None] * P)) ** 2, axis=0)
        sq[i] = np.sqrt(ora.blur_periodic(i_mod, g) if sigma > 0 else i_mod)
    return O, P, positions, params, sq


def test_consistent_data_is_a_fixed_point(rng):
    for sigma, dom in ((0.0, ora.BLUR_AMPLITUDE), (1.2, ora.BLUR_INTENSITY)):
        O, P, positions, params, sq = _consistent(rng, sigma=sigma, blur_domain=dom)
        params.eps = 0.0
        st, errs = pclsqml.iterate(ora.State(O=O, P=P), None, positions, params, 1, sqrt_I=sq)
        np.testing.assert_allclose(st.O, O, atol=1e-10)
        np.testing.assert_allclose(st.P, P, atol=1e-10)
        assert errs[0] < 1e-18


def test_single_position_object_step_lands_on_the_modulus_projection(rng):
    # one box, K = 1, probe frozen, no blur, gamma_obj = 0 (dO = chi / P) and no damping:
    # the optimal object step is 1 and the new exit wave is the Fourier-modulus projection
    n = 8
    O = _cplx(rng, n, n)
    P = (1.0 + rng.random((1, n, n))) * np.exp(1j * rng.standard_normal((1, n, n)))
    sq = rng.random((1, n, n)) + 0.5
    params = ora.Params(n=n, sigma1=0.0, sigma2=0.0, kernel_size=1, eps=0.0, probe_update_start=10,
                        gamma_obj=0.0)
    O_new, P_new, _, cap = pclsqml.batch_step(O, P, sq, np.array([(0, 0)]), [0], 1, params, lam=0.0, capture=True)
    assert abs(cap["steps"][0, 0] - 1.0) < 1e-12 and cap["steps"][0, 1] == 0.0
    assert P_new is P
    Psi = np.fft.fft2(O_new * P[0], norm="ortho")
    np.testing.assert_allclose(np.abs(Psi), sq[0], atol=1e-12)
    Psi0 = np.fft.fft2(O * P[0], norm="ortho")
    np.testing.assert_allclose(np.angle(Psi), np.angle(Psi0), atol=1e-9)


def test_single_position_object_and_probe_steps_closed_form(rng):
    # one box, K = 1, no blur, gamma = 0 for both (dO = chi / P, dP = chi / o): both
    # directions change the exit wave by chi, so the damped normal equations are
    # |chi|^2 [[1 + lam, 1], [1, 1 + lam]] [a, b] = |chi|^2 [1, 1], i.e. a = b = 1 / (2 + lam)
    n, lam = 8, 0.3
    O = (1.0 + rng.random((n, n))) * np.exp(1j * rng.standard_normal((n, n)))
    P = (1.0 + rng.random((1, n, n))) * np.exp(1j * rng.standard_normal((1, n, n)))
    sq = rng.random((1, n, n)) + 0.5
    params = ora.Params(n=n, sigma1=0.0, sigma2=0.0, kernel_size=1, eps=0.0, gamma_obj=0.0, gamma_probe=0.0)
    O_new, P_new, _, cap = pclsqml.batch_step(O, P, sq, np.array([(0, 0)]), [0], 1, params, lam=lam, capture=True)
    np.testing.assert_allclose(cap["steps"][0], [1 / (2 + lam)] * 2, rtol=1e-12)
    chi = cap["chi"][0, 0]
    np.testing.assert_allclose(O_new, O + chi / P[0] / (2 + lam), atol=1e-12)
    np.testing.assert_allclose(P_new[0], P[0] + chi / O / (2 + lam), atol=1e-12)


def test_batch_moves_by_the_mean_step(rng):
    # two positions: the object moves by obj_step times the mean of the two positions'
    # object steps along the batch direction N_O / ((1 - g) W + g max W)
    O, P, positions, params, sq = _consistent(rng, k=1)
    sq = sq * (1.0 + 0.2 * rng.random(sq.shape))  # inconsistent data: nonzero updates
    params.obj_step, params.probe_step = 0.7, 0.4
    O_new, P_new, _, cap = pclsqml.batch_step(O, P, sq, positions, [3, 9], 1, params, lam=0.1, capture=True)
    n = params.n
    w = np.zeros(O.shape)
    for j in (3, 9):
        r, c = positions[j]
        w[r:r + n, c:c + n] += np.abs(P[0]) ** 2
    m = cap["mask"]
    dO = cap["n_o"][m] / (0.8 * w[m] + 0.2 * w.max())
    np.testing.assert_allclose(O_new[m], O[m] + 0.7 * np.mean(cap["steps"][:, 0]) * dO, atol=1e-13)
    np.testing.assert_array_equal(O_new[~m], O[~m])
    np.testing.assert_allclose(P_new, P + 0.4 * np.mean(cap["steps"][:, 1]) * cap["dP"], atol=1e-13)


def test_noise_free_convergence():
    import datagen
    spec = dict(datagen.CONFIGS["far64"])
    spec.update(obj=(48, 48), n=16, n_side=4, step=6, radius=5, jitter=0, sigma_data=0.0)
    s = datagen.make_scan(spec, 5, noise=False, probe_known=True)
    params = ora.Params(n=16, sigma1=0.0, sigma2=0.0, kernel_size=1, probe_update_start=1000, batch=4,
                        gamma_obj=0.1)
    roi = ora.illumination_roi(s["positions"], s["probe_true"], s["obj_true"].shape)
    st = ora.State(O=s["obj0"], P=s["probe0"])
    e0 = ora.nmse(st.O, s["obj_true"], roi)
    st, errs = pclsqml.iterate(st, s["intensities"], s["positions"], params, 60)
    e1 = ora.nmse(st.O, s["obj_true"], roi)
    assert e1 < 1e-3 and e1 < 0.01 * e0
    assert errs[-1] < 0.01 * errs[0]
