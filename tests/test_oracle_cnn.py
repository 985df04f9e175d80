"""Pins for the FP64 warm-start network: convolution against scipy's
correlation, and the analytic gradient against central finite differences."""

import numpy as np
import scipy.signal

from oracle import cnn


def test_conv_matches_scipy_correlation(rng):
    x = rng.standard_normal((2, 3, 11, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv_forward(x, w, b, 1)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(x[n, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[n, o], ref, atol=1e-12)
    y2 = cnn.conv_forward(x, w, b, 2)
    np.testing.assert_allclose(y2, y[:, :, ::2, ::2], atol=1e-12)
    assert y2.shape == (2, 4, 6, 5)


def test_gradient_matches_finite_differences(rng):
    layers = [(1, 3, 2), (3, 4, 2), (4, 4, 1)]
    theta = cnn.init_params(rng, layers, 2)
    x = rng.standard_normal((3, 1, 12, 12))
    t = rng.standard_normal((3, 2))
    loss, g = cnn.loss_and_grad(theta, x, t, layers, 2)
    idx = rng.choice(theta.size, 40, replace=False)
    h = 1e-6
    num = []
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        num.append((cnn.loss_and_grad(tp, x, t, layers, 2)[0] - cnn.loss_and_grad(tm, x, t, layers, 2)[0]) / (2 * h))
    num = np.array(num)
    np.testing.assert_allclose(g[idx], num, rtol=1e-6, atol=1e-9)
    assert loss > 0


def test_shapes_and_count():
    assert cnn.param_count() == 32 * 9 + 32 + 5 * (32 * 32 * 9 + 32) + 4 * 32 + 4
    rng = np.random.default_rng(0)
    theta = cnn.init_params(rng)
    y, (acts, feat) = cnn.forward(theta, rng.standard_normal((1, 1, 128, 128)))
    assert y.shape == (1, 4)
    assert [a.shape[2] for a in acts] == [128, 64, 32, 16, 8, 4, 4]


def test_bf16_round_values():
    # exactly representable values are kept; ties go to the even mantissa
    v = np.array([1.0, -2.5, 0.0, 3.140625, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9])
    np.testing.assert_array_equal(cnn.bf16_round(v), [1.0, -2.5, 0.0, 3.140625, 1.0, 1.0 + 2.0 ** -6, 1.0])
    r = np.random.default_rng(3).standard_normal(1000)
    q = cnn.bf16_round(r)
    assert np.all(np.abs(q - r) <= np.abs(r) * 2.0 ** -8)
    np.testing.assert_array_equal(cnn.bf16_round(q), q)


def test_rounded_activations_reduce_to_plain_network(rng):
    layers = [(1, 3, 2), (3, 4, 2), (4, 4, 1)]
    theta = cnn.init_params(rng, layers, 2)
    x = rng.standard_normal((2, 1, 12, 12))
    t = rng.standard_normal((2, 2))
    l0, g0 = cnn.loss_and_grad(theta, x, t, layers, 2)
    l1, g1 = cnn.loss_and_grad(theta, x, t, layers, 2, act_round=lambda a: a)
    assert l0 == l1 and np.array_equal(g0, g1)
    l2, g2 = cnn.loss_and_grad(theta, x, t, layers, 2, act_round=cnn.bf16_round)
    assert abs(l2 - l0) < 1e-2 * l0
