"""A warm-start network whose ReLU decisions cannot flip under rounding.

With random weights some pre-activations lie within rounding distance of zero,
so a network that stores its activations in BF16 takes a few ReLU decisions
differently from an FP64 one and the two gradients differ by whole pixels.
margin_network sets each channel's bias so that every pre-activation of that
channel over the given batch is at least delta away from zero (half of the
channels always on, half always off), with delta a quarter of the channel's
spread of pre-bias sums -- far above the BF16 storage error -- so an FP64
network and a lower-precision one make identical ReLU decisions."""

from __future__ import annotations

import numpy as np

from oracle import cnn


def margin_network(rng, x, layers=cnn.LAYERS, n_out=cnn.N_OUT, bf16_weights=False):
    """(theta, [delta per layer, per channel]) for the batch x [nb, 1, H, W]."""
    theta = cnn.init_params(rng, layers, n_out)
    if bf16_weights:
        o = 0
        for ci, co, _ in layers:
            theta[o:o + co * ci * 9] = cnn.bf16_round(theta[o:o + co * ci * 9])
            o += co * ci * 9 + co
        theta[o:o + n_out * layers[-1][1]] = cnn.bf16_round(theta[o:o + n_out * layers[-1][1]])
    theta[-n_out:] = 0.1 * rng.standard_normal(n_out)
    convs, _ = cnn.unpack(theta, layers, n_out)
    a = x
    o = 0
    deltas = []
    for (w, _), (ci, co, s) in zip(convs, layers):
        pre = cnn.conv_forward(a, w, np.zeros(co), s)
        lo = pre.min(axis=(0, 2, 3))
        hi = pre.max(axis=(0, 2, 3))
        delta = 0.25 * np.maximum(hi - lo, 1e-3)
        on = rng.permutation(co) < (co + 1) // 2
        b = np.where(on, delta - lo, -hi - delta)
        if bf16_weights:  # biases are held in float32
            b = b.astype(np.float32).astype(np.float64)
        theta[o + co * ci * 9:o + co * ci * 9 + co] = b
        o += co * ci * 9 + co
        deltas.append(np.minimum(np.where(on, lo + b, -(hi + b)), delta))
        a = np.maximum(pre + b[None, :, None, None], 0.0)
    return theta, deltas
