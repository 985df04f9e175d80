"""Pins of the FP64 CGLS monochromatisation (oracle/mono.py, Sec. 4.2, Eq. 12-13):
the broadband operator against its definition on smooth patterns (direction of the
magnification, power per wavelength), CGLS against the dense least-squares
solution, its iterates against the Krylov subspace of Eq. 13, and its residuals."""

import numpy as np

from oracle import mono

SCALES = [1.0 / (1.0 + s) for s in (-0.025, -0.0125, 0.0, 0.0125, 0.025)]


def _gauss(n, sig, cy=None, cx=None):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    cy = n / 2 if cy is None else cy
    cx = n / 2 if cx is None else cx
    return np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * sig * sig))


def test_monochromatic_operator_is_identity():
    op = mono.broadband_operator(16, [1.0], [1.0])
    m = np.random.default_rng(0).random((16, 16))
    np.testing.assert_allclose(mono.apply_C(op, m), m, atol=1e-14)


def test_magnification_of_a_smooth_pattern():
    # one wavelength with s = lambda_c / lambda = 1.1: the pattern is m(c + s (u - c)) s^2, i.e. a
    # centred Gaussian of width sigma becomes one of width sigma / s with peak s^2 (bilinear
    # sampling of a smooth function: error well below 1e-2 of the peak)
    n, sig, s = 64, 6.0, 1.1
    op = mono.broadband_operator(n, [s], [1.0])
    got = mono.apply_C(op, _gauss(n, sig))
    ref = s * s * _gauss(n, sig / s)
    assert np.max(np.abs(got - ref)) < 1e-2 * ref.max()
    # power of each wavelength is its weight (pattern inside the frame); bilinear sampling of a
    # curved profile biases the sum by O(1 / sigma^2) of a pixel: ~1e-3 at sigma = 5
    op = mono.broadband_operator(n, SCALES, [1, 2, 3, 2, 1])
    m = _gauss(n, 5.0)
    assert abs(mono.apply_C(op, m).sum() / m.sum() - 1.0) < 3e-3
    # a wrong magnification direction (s -> 1 / s) or a missing s^2 fails the width check above:
    wrong = mono.apply_C(mono.broadband_operator(n, [1 / s], [1.0]), _gauss(n, sig)) * s ** 4
    assert np.max(np.abs(wrong - ref)) > 0.1 * ref.max()


def test_adjoint():
    rng = np.random.default_rng(1)
    op = mono.broadband_operator(12, SCALES, [1] * 5)
    x, y = rng.random((12, 12)), rng.random((12, 12))
    assert abs(np.sum(mono.apply_C(op, x) * y) - np.sum(x * mono.apply_CT(op, y))) < 1e-12


def _dense(op, n):
    A = np.zeros((n * n, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        A[:, j] = mono.apply_C(op, e.reshape(n, n)).ravel()
    return A


def test_cgls_reaches_least_squares_and_stays_in_krylov_space():
    n = 8
    rng = np.random.default_rng(2)
    op = mono.broadband_operator(n, [0.8, 1.0, 1.25], [1, 1, 1])
    b = rng.random((n, n))
    A = _dense(op, n)
    ref, *_ = np.linalg.lstsq(A, b.ravel(), rcond=None)
    x, res = mono.cgls(op, b, n * n)
    np.testing.assert_allclose(x.ravel(), ref, atol=1e-8 * np.abs(ref).max())
    # residuals never increase (CGLS minimises ||C x - b|| over nested Krylov spaces)
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))
    # x_k lies in span{C^T b, (C^T C) C^T b, ..., (C^T C)^(k-1) C^T b}  (Eq. 13)
    k = 4
    xk, _ = mono.cgls(op, b, k)
    v = A.T @ b.ravel()
    basis = [v]
    for _ in range(k - 1):
        v = A.T @ (A @ v)
        basis.append(v)
    Bm = np.stack(basis, axis=1)
    coef, *_ = np.linalg.lstsq(Bm, xk.ravel(), rcond=None)
    assert np.linalg.norm(Bm @ coef - xk.ravel()) < 1e-8 * np.linalg.norm(xk)
    # and it is the best point of that space: the residual equals the projected least squares
    c2, *_ = np.linalg.lstsq(A @ Bm, b.ravel(), rcond=None)
    assert abs(np.linalg.norm(A @ Bm @ c2 - b.ravel()) - np.linalg.norm(A @ xk.ravel() - b.ravel())) < 1e-8


def test_consistent_broadband_data_is_recovered():
    # b = C m for a pattern well inside the frame and the 5-wavelength +-2.5 % spectrum:
    # 25 iterations (the paper's optimum k) recover m closely
    n = 64
    m = _gauss(n, 4.0) + 0.5 * _gauss(n, 2.0, 20, 40)
    op = mono.broadband_operator(n, SCALES, [1] * 5)
    x, res = mono.cgls(op, mono.apply_C(op, m), 25)
    assert np.linalg.norm(x - m) < 2e-2 * np.linalg.norm(m)
    assert res[-1] < 1e-3 * res[0]
