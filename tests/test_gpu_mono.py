"""GPU CGLS monochromatisation (ptycho_mono_*, Sec. 4.2, Eq. 12-13) against the FP64
oracle (oracle/mono.py): the iterate after k = 25 iterations (the paper's usual k) and
the residual history, for the 5-wavelength +-2.5 % spectrum of the 1024^2-object
workload at 64^2 and 256^2 frames and a wide 3-line spectrum, through the C ABI.

Bar: relative L2 <= 1e-5 of the iterate, and every residual within 1e-5 of the
data norm |b| (a small late residual is a difference of FP32 vectors, so its own
relative error is larger).  CGLS on a well-conditioned C (magnifications a few
per cent apart) does not amplify the FP32 rounding of its vectors beyond that;
the scalars alpha, beta and the residual sums are accumulated in double.  For a
wide spectrum the bar scales with the conditioning: CGLS runs conjugate gradients
on the normal equations, whose condition number is kappa(C)^2, and rounding of
order eps_32 in its vectors perturbs the iterates and the residual recurrence by
up to that factor (kappa measured on the dense operator of a 32^2 frame), so the
iterate and the residuals are held to max(1e-5, 4 kappa^2 eps_32).  The operators
themselves are pinned before any amplification by the first two iterates, at
1e-5 for every spectrum (test_cgls_first_iterates_pin_the_operators).
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import mono
from parity_util import rel_l2

pytestmark = pytest.mark.gpu

SCALES_C2 = [1.0 / (1.0 + s) for s in (-0.025, -0.0125, 0.0, 0.0125, 0.025)]


def _patterns(rng, n, count, scales, weights):
    """Broadband data b = C m of smooth random monochromatic patterns, plus 1e-3 noise."""
    y, x = np.mgrid[0:n, 0:n].astype(float)
    op = mono.broadband_operator(n, scales, weights)
    ms, bs = [], []
    for _ in range(count):
        m = np.zeros((n, n))
        for _ in range(6):
            cy, cx = rng.uniform(0.3 * n, 0.7 * n, 2)
            sig = rng.uniform(0.03, 0.1) * n
            m += rng.uniform(0.2, 1.0) * np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * sig * sig))
        b = mono.apply_C(op, m)
        b += 1e-3 * b.max() * rng.standard_normal(b.shape)
        ms.append(m)
        bs.append(b)
    return op, np.array(ms), np.array(bs)


def _kappa(n, scales, weights):
    op = mono.broadband_operator(n, scales, weights)
    A = np.zeros((n * n, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        A[:, j] = mono.apply_C(op, e.reshape(n, n)).ravel()
    sv = np.linalg.svd(A, compute_uv=False)
    return float(sv[0] / sv[-1])


@pytest.mark.parametrize("n,count,scales,weights", [
    (64, 5, SCALES_C2, [1, 1, 1, 1, 1]),
    (256, 3, SCALES_C2, [1, 2, 3, 2, 1]),
    (32, 4, [0.8, 1.0, 1.3], [0.5, 1.0, 0.7]),
])
def test_cgls_matches_oracle(n, count, scales, weights):
    import paper_2406_06640_amd as P
    print(f"\n[gpu-case] CGLS monochromatisation n={n} patterns={count} lines={len(scales)}", flush=True)
    rng = np.random.default_rng(n + count)
    op, ms, bs = _patterns(rng, n, count, scales, weights)
    k = 25
    b32 = bs.astype(np.float32)
    out = np.zeros_like(b32)
    with P.Monochromatiser(n, count, scales, weights) as mc:
        res = mc.run(b32, out, k)
        out2 = np.zeros_like(b32)
        res2 = mc.run(b32, out2, k)
    np.testing.assert_array_equal(out, out2)
    np.testing.assert_array_equal(res, res2)
    tol = 1e-5
    if scales is not SCALES_C2:
        kappa = _kappa(n, scales, weights)
        tol = max(1e-5, 4 * kappa * kappa * np.finfo(np.float32).eps)
        print(f"kappa(C) = {kappa:.1f}: iterate bar {tol:.1e}", flush=True)
    worst = 0.0
    for i in range(count):
        x, r = mono.cgls(op, b32[i].astype(np.float64), k)
        ex = rel_l2(out[i], x)
        er = float(np.max(np.abs(res[i] - np.array(r)))) / r[0]
        print(f"pattern {i}: iterate relative L2 {ex:.2e}, residuals {er:.2e} of |b|, "
              f"recovery |x - m| / |m| {rel_l2(out[i], ms[i]):.2e}", flush=True)
        worst = max(worst, ex)
        assert ex <= tol and er <= tol
    assert worst > 0.0  # the two sides are computed independently


@pytest.mark.parametrize("n,scales,weights", [
    (64, SCALES_C2, [1, 1, 1, 1, 1]),
    (96, [0.8, 1.0, 1.3], [0.5, 1.0, 0.7]),
    (256, [0.25, 1.0, 3.5], [1.0, 0.3, 0.2]),
])
def test_cgls_first_iterates_pin_the_operators(n, scales, weights):
    """One and two CGLS iterations: x_1 = (|C^T b|^2 / |C C^T b|^2) C^T b and its successor
    touch each operator once or twice, before the conditioning can amplify FP32 rounding,
    so they hold the operator and its adjoint to 1e-5 whatever the spectrum (the sample
    positions c + s (u - c) are FP32 on the GPU: about 1e-6 relative for scales that are
    not exactly representable).  The third spectrum's magnifications differ 14-fold, so
    the input regions of some output tiles exceed LDS and take the global-memory path."""
    import paper_2406_06640_amd as P
    print(f"\n[gpu-case] CGLS first iterates n={n} lines={len(scales)}", flush=True)
    rng = np.random.default_rng(7 + n)
    op, _, bs = _patterns(rng, n, 3, scales, weights)
    b32 = bs.astype(np.float32)
    with P.Monochromatiser(n, 3, scales, weights) as mc:
        for k in (1, 2):
            out = np.zeros_like(b32)
            mc.run(b32, out, k)
            for i in range(3):
                x, _ = mono.cgls(op, b32[i].astype(np.float64), k)
                err = rel_l2(out[i], x)
                print(f"k={k} pattern {i}: relative L2 {err:.2e}", flush=True)
                assert err <= 1e-5


def test_cgls_zero_iterations_and_zero_data():
    import paper_2406_06640_amd as P
    n = 32
    b = np.zeros((2, n, n), np.float32)
    b[1, 10, 12] = 1.0
    out = np.ones_like(b)
    with P.Monochromatiser(n, 4, SCALES_C2, [1] * 5) as mc:
        res = mc.run(b, out, 0)
        assert np.all(out == 0) and res.shape == (2, 1)
        assert res[0, 0] == 0 and abs(res[1, 0] - 1.0) < 1e-7
        res = mc.run(b, out, 3)
        assert np.all(out[0] == 0) and np.all(res[0] == 0)
        with pytest.raises(P.PtychoError):
            mc.run(np.zeros((5, n, n), np.float32), np.zeros((5, n, n), np.float32), 3)
