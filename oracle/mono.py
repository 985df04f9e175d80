"""Plain FP64 numerical monochromatisation by CGLS (test infrastructure only).

Sec. 4.2 of the paper: a broadband far-field pattern b is modelled as b = C m,
with m the monochromatic pattern and C a matrix that depends only on the
source spectrum; m is recovered by CGLS, the k-th iterate being the
least-squares solution of ||C x - b|| over the Krylov subspace
kappa_k = span{C^T b, (C^T C) C^T b, ..., (C^T C)^(k-1) C^T b} (Eq. 12-13).

Reading of C (the paper gives no formula): on a fixed detector the pattern at
wavelength lambda_j samples the scattering spectrum at spatial frequencies
scaled by s_j = lambda_c / lambda_j, so the pattern at lambda_j is m magnified
about the centre pixel c = N / 2: m(c + s_j (u - c)), times s_j^2 so that each
wavelength carries the power of its weight w_j (sum_j w_j = 1).  Sampling
between pixels is bilinear, samples outside the frame are zero, and the
operator is separable:  C m = sum_j w_j s_j^2 S_j m S_j^T  with S_j the 1D
N x N interpolation matrix of scale s_j.  The object's own dispersion is not
part of C (the method's assumption).

CGLS is written in its textbook form (Hestenes and Stiefel's conjugate
gradients on the normal equations, as in Bjorck's CGLS), started at x_0 = 0.
"""

from __future__ import annotations

import math

import numpy as np


def interp_matrix(n, s):
    """S[u, v]: weight of detector pixel v in the value sampled at c + s (u - c), c = n / 2
    (bilinear in 1D: weight 1 - |p - v| for |p - v| < 1, samples outside [0, n) are zero)."""
    c = n / 2
    S = np.zeros((n, n))
    for u in range(n):
        p = c + s * (u - c)
        i0 = math.floor(p)
        t = p - i0
        if 0 <= i0 < n:
            S[u, i0] += 1.0 - t
        if 0 <= i0 + 1 < n and t > 0:
            S[u, i0 + 1] += t
    return S


def broadband_operator(n, scales, weights):
    """[(w_j s_j^2, S_j)] for the spectrum (scales s_j = lambda_c / lambda_j, weights w_j)."""
    w = np.asarray(weights, dtype=np.float64)
    w = w / w.sum()
    return [(wj * sj * sj, interp_matrix(n, sj)) for sj, wj in zip(scales, w)]


def apply_C(op, m):
    """C m = sum_j w_j s_j^2 S_j m S_j^T."""
    out = np.zeros_like(m, dtype=np.float64)
    for a, S in op:
        out += a * (S @ m @ S.T)
    return out


def apply_CT(op, r):
    """C^T r = sum_j w_j s_j^2 S_j^T r S_j."""
    out = np.zeros_like(r, dtype=np.float64)
    for a, S in op:
        out += a * (S.T @ r @ S)
    return out


def cgls(op, b, k_iters):
    """k_iters CGLS iterations for min ||C x - b|| from x_0 = 0.  Returns (x_k, [||C x_i - b|| for i = 0..k])."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    s = apply_CT(op, r)
    p = s.copy()
    gamma = float(np.sum(s * s))
    res = [float(np.linalg.norm(r))]
    for _ in range(k_iters):
        if gamma == 0.0:
            res.append(res[-1])
            continue
        q = apply_C(op, p)
        alpha = gamma / float(np.sum(q * q))
        x = x + alpha * p
        r = r - alpha * q
        s = apply_CT(op, r)
        gamma_new = float(np.sum(s * s))
        beta = gamma_new / gamma
        p = s + beta * p
        gamma = gamma_new
        res.append(float(np.linalg.norm(r)))
    return x, res
