"""GPU checks of the learned warm start against the FP64 references in
oracle/cnn.py and oracle/forward_model.py: network loss, gradient and
prediction (BF16 weights and activations, FP32 accumulation), the input
features, the rendered probe, the forward-model patterns, the generator's
determinism and ranges, and that training on generated data lowers the loss."""

from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import cnn
from oracle import forward_model as fm
from parity_util import make_case, rel_l2

pytestmark = pytest.mark.gpu

# BF16 weights and BF16-stored activations (8 significant bits) with FP32 sums:
# a few 2^-9 relative roundings per layer, compounded over six layers and the
# backward pass.  The gradient is compared with the all-FP64 network on a batch
# whose pre-activations all stay a margin away from zero (tests/cnn_util.py), so
# both take the same ReLU decisions and only the rounding differs.
GRAD_TOL = 2e-2
# Adam in FP32 against FP64: the update lr m^/(sqrt(v^) + eps) is a handful of
# roundings per element (~1e-7 relative) plus the rounding of theta itself to
# float32 (half an ulp of |theta| ~ 0.5, i.e. ~3e-8, against steps of lr = 1e-2).
ADAM_TOL = 1e-5
PRED_TOL = 2e-2


def _announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _bf16_weights(theta):
    """Round the weights (not the biases) of a parameter vector to BF16."""
    t = np.asarray(theta, dtype=np.float32).copy()
    o = 0
    for ci, co, _ in cnn.LAYERS:
        t[o:o + co * ci * 9] = cnn.bf16_round(t[o:o + co * ci * 9]).astype(np.float32)
        o += co * ci * 9 + co
    t[o:o + cnn.N_OUT * 32] = cnn.bf16_round(t[o:o + cnn.N_OUT * 32]).astype(np.float32)
    return t


def _layer_slices():
    out, o = [], 0
    for i, (ci, co, _) in enumerate(cnn.LAYERS):
        out.append((f"conv{i + 1}.w", slice(o, o + co * ci * 9)))
        o += co * ci * 9
        out.append((f"conv{i + 1}.b", slice(o, o + co)))
        o += co
    out.append(("head.w", slice(o, o + cnn.N_OUT * 32)))
    out.append(("head.b", slice(o + cnn.N_OUT * 32, o + cnn.N_OUT * 33)))
    return out


def _inputs(rng, nb):
    # smooth-ish standardised images, zero border like the real features
    x = np.zeros((nb, 128, 128))
    core = rng.standard_normal((nb, 64, 64))
    k = np.ones(5) / 5.0
    core = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), 2, core)
    core = (core - core.mean(axis=(1, 2), keepdims=True)) / core.std(axis=(1, 2), keepdims=True)
    x[:, 32:96, 32:96] = core
    return x


def _margin_case(nb=16, seed=2024):
    from cnn_util import margin_network
    rng = np.random.default_rng(seed)
    x = _inputs(rng, nb).astype(np.float32).astype(np.float64)
    theta, _ = margin_network(rng, x[:, None], bf16_weights=True)
    theta = theta.astype(np.float32)
    t = rng.standard_normal((nb, 4)).astype(np.float32).astype(np.float64)
    return theta, x, t


def test_network_loss_and_gradient_match_fp64():
    """Loss and gradient of a 16-sample batch against the all-FP64 network (BF16
    weights, FP64 everything else), ReLU decisions made safe by the margin construction."""
    import torch
    from paper_2406_06640_amd.learned import WarmStartNet
    _announce("network loss/gradient nb=16 vs FP64 oracle (margin network)")
    theta, x, t = _margin_case()
    loss_ref, g_ref = cnn.loss_and_grad(theta.astype(np.float64), x[:, None], t)
    with WarmStartNet(max_batch=16, params=theta, normalise=False) as net:
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        td = torch.from_numpy(t.astype(np.float32)).cuda()
        loss, g = net.loss_grad(xd, td)
        loss2, g2 = net.loss_grad(xd, td)
    assert loss == loss2 and np.array_equal(g, g2), "gradients are not reproducible"
    err = rel_l2(g.astype(np.float64), g_ref)
    per = {name: rel_l2(g[s].astype(np.float64), g_ref[s]) for name, s in _layer_slices()}
    print(f"loss {loss:.6f} vs {loss_ref:.6f}; gradient relative L2 {err:.2e}", flush=True)
    print("per block:", {k: f"{v:.1e}" for k, v in per.items()}, flush=True)
    assert abs(loss - loss_ref) / loss_ref < PRED_TOL
    assert err < GRAD_TOL
    for name, v in per.items():
        # the bias gradients of always-off channels are exactly zero on both sides
        assert v < 5 * GRAD_TOL, (name, v)


def test_adam_steps_match_fp64():
    """Two ptycho_ws_train_step calls against the FP64 Adam update (Kingma and Ba) fed
    with the gradient the library computes at the same point."""
    import torch
    from paper_2406_06640_amd.learned import WarmStartNet
    _announce("two Adam steps vs FP64 Adam")
    theta, x, t = _margin_case(nb=8, seed=77)
    lr = 1e-2
    with WarmStartNet(max_batch=8, params=theta, normalise=False) as net:
        net.reset_optimizer()
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        td = torch.from_numpy(t.astype(np.float32)).cuda()
        th = theta.astype(np.float64)
        m = np.zeros_like(th)
        v = np.zeros_like(th)
        for step in (1, 2):
            _, g = net.loss_grad(xd, td)
            net.train_step(xd, td, lr=lr)
            got = net.get_params().astype(np.float64)
            ref, m, v = cnn.adam_step(th, g.astype(np.float64), m, v, step, lr)
            err = rel_l2(got - th, ref - th)
            # per element: the update's own error plus the float32 rounding of theta
            bound = ADAM_TOL * lr + 2.0 ** -23 * np.abs(ref)
            worst = float(np.max(np.abs(got - ref) / bound))
            print(f"step {step}: update relative L2 {err:.2e}, worst element at {worst:.2f} of its bound",
                  flush=True)
            assert err < ADAM_TOL
            assert worst <= 1.0
            th = got


def test_prediction_matches_fp64_with_target_scaling():
    import torch
    from paper_2406_06640_amd import learned as L
    _announce("network prediction nb=5 (natural units)")
    rng = np.random.default_rng(7)
    theta = _bf16_weights(cnn.init_params(rng))
    x = _inputs(rng, 5).astype(np.float32).astype(np.float64)
    y_ref, _ = cnn.forward(theta.astype(np.float64), x[:, None])
    y_ref = y_ref * np.array(L.TARGET_SCALE) + np.array(L.TARGET_OFFSET)
    idx = torch.tensor([4, 0, 2], dtype=torch.int32, device="cuda")
    with L.WarmStartNet(max_batch=8, params=theta) as net:
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        y = net.forward(xd).cpu().numpy()
        y_idx = net.forward(xd, idx=idx).cpu().numpy()
    err = rel_l2(y.astype(np.float64), y_ref)
    print(f"prediction relative L2 {err:.2e}", flush=True)
    assert err < PRED_TOL
    np.testing.assert_array_equal(y_idx, y[[4, 0, 2]])


def test_features_match_oracle():
    import torch
    from paper_2406_06640_amd.learned import ptycho_ws_features
    _announce("features of a 64x64 scan")
    s = make_case(n=64, k=1, obj=(144, 144), n_side=10, step=8, radius=16, seed=5)
    ints = s["intensities"]
    got = ptycho_ws_features(torch.from_numpy(ints).cuda()).cpu().numpy()
    ref = fm.features(ints, 128)
    print(f"features max abs error {np.max(np.abs(got - ref)):.2e}", flush=True)
    np.testing.assert_allclose(got, ref, atol=2e-4)
    flat = ptycho_ws_features(torch.full((3, 32, 32), 4.0, device="cuda")).cpu().numpy()
    assert np.all(flat == 0)


@pytest.mark.parametrize("n,k,radius,defocus", [(64, 4, 15.5, 1.3), (64, 1, 12.0, 0.5), (128, 3, 40.0, 2.0)])
def test_render_probe_matches_oracle(n, k, radius, defocus):
    from paper_2406_06640_amd.learned import ptycho_ws_render_probe
    _announce(f"render probe n={n} K={k}")
    got = ptycho_ws_render_probe(n, k, radius, defocus, 1234.5).cpu().numpy()
    ref = fm.render_probe(n, k, radius, defocus, 1234.5)
    err = rel_l2(got, ref)
    print(f"probe relative L2 {err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("sigma,bw,radius,defocus", [(1.7, 0.04, 15.0, 1.3), (0.5, 0.0, 19.5, 0.6), (3.0, 0.02, 12.0, 2.0)])
def test_forward_model_patterns_match_oracle(sigma, bw, radius, defocus):
    import torch
    from paper_2406_06640_amd.learned import ForwardModel
    _announce(f"forward-model patterns sigma={sigma} bw={bw}")
    rng = np.random.default_rng(11)
    side = 144
    la = np.log(0.8 + 0.2 * rng.random((side, side)))
    ph = rng.uniform(-math.pi / 2, math.pi / 2, (side, side))
    pos = np.array([[0, 0], [40, 17], [80, 80]], dtype=np.int32)
    obj = torch.from_numpy(np.stack([la, ph], axis=-1).astype(np.float32)).cuda()
    with ForwardModel(max_chunk=1) as g:
        got = g.patterns(obj, pos, sigma, bw, radius, defocus).cpu().numpy()
        with pytest.raises(Exception):
            g.patterns(obj, np.array([[81, 0]], dtype=np.int32), sigma, bw, radius, defocus)
    probe = fm.aperture(64, radius, defocus)
    probe = probe / math.sqrt(np.sum(np.abs(probe) ** 2))
    scales = fm.wavelength_scales(bw)
    for i, (r, c) in enumerate(pos):
        ref = fm.farfield_pattern(la[r:r + 64, c:c + 64].astype(np.float32).astype(np.float64),
                                  ph[r:r + 64, c:c + 64].astype(np.float32).astype(np.float64), probe, scales, sigma)
        err = rel_l2(got[i], ref)
        print(f"position {i}: relative L2 {err:.2e}", flush=True)
        assert err < 1e-4


def test_generator_ranges_and_determinism():
    from paper_2406_06640_amd import learned as L
    _announce("generator 8 samples, chunked twice")
    with L.ForwardModel(max_chunk=8) as g:
        f8, t8 = g.generate(99, 100, 8)
        f4, t4 = g.generate(99, 104, 4)
        obj = g.objects(99, 100, 2).cpu().numpy()
    f8, t8, f4, t4 = (a.cpu().numpy() for a in (f8, t8, f4, t4))
    np.testing.assert_array_equal(f8[4:], f4)
    np.testing.assert_array_equal(t8[4:], t4)
    for j, (lo, hi) in enumerate(L._RANGES):
        assert np.all(t8[:, j] >= lo) and np.all(t8[:, j] <= hi)
    core = f8[:, 32:96, 32:96]
    assert np.allclose(core.mean(axis=(1, 2)), 0, atol=1e-4)
    assert np.allclose(core.std(axis=(1, 2)), 1, atol=1e-3)
    assert np.all(f8[:, :32] == 0) and np.all(f8[:, :, 96:] == 0)
    la, ph = obj[..., 0], obj[..., 1]
    assert abs(la.min() - math.log(0.8)) < 1e-6 and abs(la.max()) < 1e-6
    assert abs(ph.min() + math.pi / 2) < 1e-5 and abs(ph.max() - math.pi / 2) < 1e-5
    # the features carry the blur: wider blur, smoother mean log-pattern
    assert len(np.unique(t8[:, 0])) == 8


def test_training_lowers_the_loss():
    import torch
    from paper_2406_06640_amd import learned as L
    _announce("train 400 steps on 1024 generated samples")
    n_train, n_val = 1024, 128
    with L.ForwardModel(max_chunk=256) as g:
        feat = torch.empty((n_train + n_val, 128, 128), device="cuda")
        targ = torch.empty((n_train + n_val, 4), device="cuda")
        for s0 in range(0, n_train + n_val, 256):
            c = min(256, n_train + n_val - s0)
            g.generate(5, s0, c, feat[s0:s0 + c], targ[s0:s0 + c])
    rng = np.random.default_rng(0)
    with L.WarmStartNet(max_batch=128, params=cnn.init_params(rng).astype(np.float32)) as net:
        val_idx = torch.arange(n_train, n_train + n_val, dtype=torch.int32, device="cuda")
        loss0, _ = net.loss_grad(feat, targ, idx=val_idx)
        for step in range(400):
            idx = torch.from_numpy(rng.choice(n_train, 64, replace=False).astype(np.int32)).cuda()
            net.train_step(feat, targ, idx=idx, lr=2e-3)
        loss1, _ = net.loss_grad(feat, targ, idx=val_idx)
    print(f"validation loss {loss0:.3f} -> {loss1:.3f}", flush=True)
    assert loss1 < 0.75 * loss0
