"""FP64 reference of the warm-start network (test infrastructure only).

The network maps the mean log-intensity of a scan's patterns (a 128 x 128
image) to a few reconstruction settings (the Gaussian blur width of Eq. 7, the
source bandwidth and the probe's aperture radius and defocus).  Six 3 x 3
convolutions with 32 channels (zero padding 1; strides 2, 2, 2, 2, 2, 1; ReLU
after each), a global average pool and a linear head.  Tensors are NCHW.

Parameters are one flat vector, per convolution W[Co][Ci][3][3] then b[Co],
then the head W[T][32] and b[T].  The loss is the mean squared error over the
batch and the T outputs.  Written with plain loops over the 3 x 3 taps and
numpy for the channel sums, so it can be checked by eye and against central
finite differences.  The optimiser step is Adam (Kingma and Ba, ICLR 2015,
Algorithm 1), written out in FP64.
"""

from __future__ import annotations

import numpy as np

LAYERS = [(1, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 1)]
N_OUT = 4
INPUT = 128


def param_count(layers=LAYERS, n_out=N_OUT):
    n = 0
    for ci, co, _ in layers:
        n += co * ci * 9 + co
    return n + n_out * layers[-1][1] + n_out


def unpack(theta, layers=LAYERS, n_out=N_OUT):
    out = []
    o = 0
    for ci, co, _ in layers:
        w = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((w, b))
    c = layers[-1][1]
    hw = theta[o:o + n_out * c].reshape(n_out, c)
    o += n_out * c
    hb = theta[o:o + n_out]
    return out, (hw, hb)


def conv_forward(x, w, b, stride):
    """y[n, co, i, j] = b[co] + sum_{ci,ky,kx} w[co, ci, ky, kx] x_pad[n, ci, s i + ky, s j + kx]."""
    nb, ci, h, wd = x.shape
    co = w.shape[0]
    ho = (h - 1) // stride + 1
    wo = (wd - 1) // stride + 1
    xp = np.zeros((nb, ci, h + 2, wd + 2))
    xp[:, :, 1:h + 1, 1:wd + 1] = x
    y = np.zeros((nb, co, ho, wo)) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + stride * (ho - 1) + 1:stride, kx:kx + stride * (wo - 1) + 1:stride]
            y += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], patch)
    return y


def conv_backward(x, w, stride, dy):
    """Gradients of conv_forward: (dx, dw, db)."""
    nb, ci, h, wd = x.shape
    ho, wo = dy.shape[2], dy.shape[3]
    xp = np.zeros((nb, ci, h + 2, wd + 2))
    xp[:, :, 1:h + 1, 1:wd + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(None), slice(ky, ky + stride * (ho - 1) + 1, stride),
                  slice(kx, kx + stride * (wo - 1) + 1, stride))
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dy, xp[sl])
            dxp[sl] += np.einsum("oc,nohw->nchw", w[:, :, ky, kx], dy)
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:h + 1, 1:wd + 1], dw, db


def bf16_round(a):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even): the
    float32 bit pattern plus 0x7FFF plus bit 16, truncated to the upper 16 bits.
    Used to give the reference the BF16 weights a network stores."""
    u = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def pre_activations(theta, x, layers=LAYERS, n_out=N_OUT):
    """The convolution outputs before each ReLU, [z_1 .. z_L]."""
    convs, _ = unpack(theta, layers, n_out)
    a = x
    zs = []
    for (w, b), (_, _, s) in zip(convs, layers):
        z = conv_forward(a, w, b, s)
        zs.append(z)
        a = np.maximum(z, 0.0)
    return zs


def forward(theta, x, layers=LAYERS, n_out=N_OUT):
    """Returns (outputs [n, T], cache)."""
    convs, (hw, hb) = unpack(theta, layers, n_out)
    acts = [x]
    for (w, b), (_, _, s) in zip(convs, layers):
        acts.append(np.maximum(conv_forward(acts[-1], w, b, s), 0.0))
    feat = acts[-1].mean(axis=(2, 3))
    y = feat @ hw.T + hb
    return y, (acts, feat)


def loss_and_grad(theta, x, target, layers=LAYERS, n_out=N_OUT):
    """Mean squared error over batch and outputs, and its gradient w.r.t. theta."""
    convs, (hw, hb) = unpack(theta, layers, n_out)
    y, (acts, feat) = forward(theta, x, layers, n_out)
    nb = x.shape[0]
    diff = y - target
    loss = float(np.mean(diff ** 2))
    dy = 2.0 * diff / diff.size
    dhw = dy.T @ feat
    dhb = dy.sum(axis=0)
    dfeat = dy @ hw
    last = acts[-1]
    da = np.broadcast_to(dfeat[:, :, None, None] / (last.shape[2] * last.shape[3]), last.shape).copy()
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        w, b = convs[li]
        s = layers[li][2]
        dz = da * (acts[li + 1] > 0)
        dx, dw, db = conv_backward(acts[li], w, s, dz)
        grads.append((dw, db))
        da = dx
    grads.reverse()
    flat = []
    for dw, db in grads:
        flat += [dw.ravel(), db.ravel()]
    flat += [dhw.ravel(), dhb.ravel()]
    del nb
    return loss, np.concatenate(flat)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) at 1-based step `step`:
      m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
      m^ = m / (1 - beta1^step),      v^ = v / (1 - beta2^step),
      theta <- theta - lr m^ / (sqrt(v^) + eps).
    Returns (theta, m, v) as new arrays."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def init_params(rng, layers=LAYERS, n_out=N_OUT):
    """He-normal convolutions, zero biases, small head."""
    parts = []
    for ci, co, _ in layers:
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)))
        parts.append(np.zeros(co))
    c = layers[-1][1]
    parts.append(rng.standard_normal(n_out * c) * np.sqrt(1.0 / c))
    parts.append(np.zeros(n_out))
    return np.concatenate(parts)
