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


def test_adam_two_steps_worked_by_hand():
    # one parameter, lr 0.1, beta1 0.9, beta2 0.999, eps 1e-8; gradients 0.5 then -1.0.
    # step 1: m = 0.05, v = 0.00025, m^ = 0.05 / 0.1 = 0.5, v^ = 0.00025 / 0.001 = 0.25,
    #         theta = 1 - 0.1 * 0.5 / (0.5 + 1e-8)              = 0.900000002
    # step 2: m = 0.045 - 0.1 = -0.055, v = 0.00024975 + 0.001 = 0.00124975,
    #         m^ = -0.055 / 0.19 = -0.28947368..., v^ = 0.00124975 / 0.001999 = 0.62518759...,
    #         theta = 0.900000002 + 0.1 * 0.28947368 / (0.79068805 + 1e-8) = 0.93661035...
    th, m, v = cnn.adam_step(np.array([1.0]), np.array([0.5]), np.zeros(1), np.zeros(1), 1, 0.1)
    np.testing.assert_allclose(m, [0.05], rtol=1e-15)
    np.testing.assert_allclose(v, [0.00025], rtol=1e-12)
    np.testing.assert_allclose(th, [0.90000000199999996], rtol=1e-15)
    th, m, v = cnn.adam_step(th, np.array([-1.0]), m, v, 2, 0.1)
    np.testing.assert_allclose(m, [-0.055], rtol=1e-14)
    np.testing.assert_allclose(v, [0.00124975], rtol=1e-12)
    np.testing.assert_allclose(th, [0.93661035424056560], rtol=1e-14)


def test_adam_constant_gradient_moves_by_lr():
    # with a constant gradient g the bias-corrected moments are exactly g and g^2 at every
    # step, so each step moves theta by lr g / (|g| + eps), i.e. lr in the direction of -g
    # (a missing or wrong bias correction breaks this in the first steps)
    g = np.array([3.0, -0.02, 1e-3])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 6):
        prev = th
        th, m, v = cnn.adam_step(th, g, m, v, step, 0.01)
        np.testing.assert_allclose(th - prev, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_margin_network_keeps_pre_activations_away_from_zero(rng):
    from cnn_util import margin_network
    layers = [(1, 4, 2), (4, 6, 2), (6, 6, 1)]
    x = rng.standard_normal((3, 1, 16, 16))
    theta, delta = margin_network(rng, x, layers, 2)
    zs = cnn.pre_activations(theta, x, layers, 2)
    for z, d in zip(zs, delta):
        assert np.all(np.abs(z) >= d[None, :, None, None] * (1 - 1e-12))
        on = np.all(z > 0, axis=(0, 2, 3))
        off = np.all(z < 0, axis=(0, 2, 3))
        assert np.all(on | off) and on.any() and off.any()
    # still a smooth function of the weights: the analytic gradient matches differences
    t = rng.standard_normal((3, 2))
    _, g = cnn.loss_and_grad(theta, x, t, layers, 2)
    for i in rng.choice(theta.size, 10, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num = (cnn.loss_and_grad(tp, x, t, layers, 2)[0] - cnn.loss_and_grad(tm, x, t, layers, 2)[0]) / (2 * h)
        assert abs(g[i] - num) <= 1e-6 * max(1.0, abs(num))
