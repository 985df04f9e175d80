"""Train the warm-start network on the GPU from forward-model samples.

    python -m paper_2406_06640_amd.train_warm_start --samples 200000 --epochs 6 \
        --out paper_2406_06640_amd/weights/warm_start.npz

Samples are drawn by the library's generator (ptycho_fm_generate): far-field
scans of the 64 x 64, 10 x 10-position recipe with blur sigma in [0.5, 3] px,
bandwidth in [0, 5] %, aperture radius in [12, 20] px and defocus
coefficient in [0.5, 2].  The last `--val` samples are held out.  Training is
Adam with a cosine learning-rate decay on mini-batches of shuffled sample
indices; every forward, backward and update runs in the library's kernels.
The output file holds the FP32 parameter vector and the validation report.
"""

from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np


def init_params(rng):
    """He-normal convolution weights, zero biases, small head (the parameter order of ptycho_ws.h)."""
    layers = [(1, 32)] + [(32, 32)] * 5
    parts = []
    for ci, co in layers:
        parts.append(rng.standard_normal(co * ci * 9) * math.sqrt(2.0 / (ci * 9)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(4 * 32) * math.sqrt(1.0 / 32))
    parts.append(np.zeros(4))
    return np.concatenate(parts).astype(np.float32)


def generate(fm, seed, n, chunk, log_every=20.0):
    import torch
    feat = torch.empty((n, 128, 128), dtype=torch.float32, device="cuda")
    targ = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    t0 = last = time.time()
    for s0 in range(0, n, chunk):
        c = min(chunk, n - s0)
        fm.generate(seed, s0, c, feat[s0:s0 + c], targ[s0:s0 + c])
        if time.time() - last > log_every:
            torch.cuda.synchronize()
            last = time.time()
            print(f"  generated {s0 + c}/{n} samples ({last - t0:.1f} s)", flush=True)
    torch.cuda.synchronize()
    return feat, targ, time.time() - t0


def evaluate(net, feat, targ, idx_all, batch):
    """Validation loss and per-target RMSE in natural units."""
    import torch
    from .learned import TARGET_NAMES
    preds = []
    for s0 in range(0, idx_all.numel(), batch):
        preds.append(net.forward(feat, idx=idx_all[s0:s0 + batch]))
    y = torch.cat(preds).double()
    t = targ[idx_all.long()].double()
    rmse = torch.sqrt(((y - t) ** 2).mean(dim=0)).cpu().numpy()
    spread = t.std(dim=0).cpu().numpy()
    return {name: dict(rmse=float(r), target_std=float(s)) for name, r, s in zip(TARGET_NAMES, rmse, spread)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--samples", type=int, default=200000)
    ap.add_argument("--val", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1005)
    ap.add_argument("--chunk", type=int, default=1024)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch
    from . import learned as L

    print(f"[train] generating {args.samples} samples on the GPU", flush=True)
    with L.ForwardModel(max_chunk=args.chunk) as fm:
        feat, targ, t_gen = generate(fm, args.seed, args.samples, args.chunk)
    print(f"[train] generation {t_gen:.1f} s ({args.samples / t_gen:.0f} samples/s)", flush=True)
    n_train = args.samples - args.val
    rng = np.random.default_rng(args.seed)
    val_idx = torch.arange(n_train, args.samples, dtype=torch.int32, device="cuda")
    steps_per_epoch = n_train // args.batch
    total = steps_per_epoch * args.epochs
    net = L.WarmStartNet(max_batch=args.batch, params=init_params(rng))
    before = evaluate(net, feat, targ, val_idx, args.batch)
    t0 = time.time()
    last = t0
    step = 0
    losses = []
    for ep in range(args.epochs):
        perm = torch.from_numpy(rng.permutation(n_train).astype(np.int32)).cuda()
        for b in range(steps_per_epoch):
            lr = 0.5 * args.lr * (1.0 + math.cos(math.pi * step / total))
            want = (b == steps_per_epoch - 1) or (time.time() - last > 15.0)
            loss = net.train_step(feat, targ, idx=perm[b * args.batch:(b + 1) * args.batch], lr=lr, want_loss=want)
            step += 1
            if want:
                last = time.time()
                losses.append((step, loss))
                print(f"  epoch {ep} step {step}/{total} loss {loss:.4f} lr {lr:.2e} ({last - t0:.1f} s)", flush=True)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    after = evaluate(net, feat, targ, val_idx, args.batch)
    vl, _ = net.loss_grad(feat, targ, idx=val_idx[:args.batch])
    report = dict(samples=args.samples, val=args.val, epochs=args.epochs, batch=args.batch, lr=args.lr,
                  seed=args.seed, steps=total, generation_s=t_gen, training_s=t_train,
                  train_samples_per_s=total * args.batch / t_train, val_loss_first_batch=vl,
                  val_before=before, val_after=after, loss_trace=losses)
    print("[train] " + json.dumps({k: v for k, v in report.items() if k != "loss_trace"}), flush=True)
    if args.out:
        np.savez(args.out, theta=net.get_params(), report=json.dumps(report))
        print(f"[train] wrote {args.out}", flush=True)
    net.close()
    return report


if __name__ == "__main__":
    main()
