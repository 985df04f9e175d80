"""The BF16 matrix-core DFT propagation path (split operands, FP32 accumulation).

Its error against the FP64 references is measured and printed per frame size;
the gates here are the stated bounds of a two-term BF16 split (each operand
carries ~16 significant bits, the dropped lo*lo term is ~2^-18 relative), not
the 1e-5 bar of the FP32 FFT path.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as ora
from parity_util import gpu_step, make_case, oracle_step, params_pair, rel_l2

pytestmark = pytest.mark.gpu

TRANSFORM_TOL = 1e-4
STEP_TOL = 1e-3


@pytest.mark.parametrize("n", [64, 128, 192, 256])
def test_dft2_bf16_matches_exact_dft(n):
    import torch
    import paper_2406_06640_amd as P
    print(f"\n[gpu-case] dft2_bf16 n={n}", flush=True)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((6, n, n)) + 1j * rng.standard_normal((6, n, n))
    t = torch.from_numpy(x.astype(np.complex64)).cuda()
    P.ptycho_dft2_bf16(t, inverse=False)
    got = t.cpu().numpy()
    ref = np.fft.fft2(x, norm="ortho")
    fwd = rel_l2(got, ref)
    P.ptycho_dft2_bf16(t, inverse=True)
    back = rel_l2(t.cpu().numpy(), x)
    print(f"n={n}: forward relative L2 {fwd:.2e}, inverse(forward) {back:.2e}", flush=True)
    assert fwd < TRANSFORM_TOL and back < 2 * TRANSFORM_TOL


@pytest.mark.parametrize("n", [64, 128, 192])
def test_dft_bf16_batch_step_error(n):
    s = make_case(n=n, k=2, obj=(n + 48, n + 48), n_side=4, step=12, radius=n // 4, seed=40 + n)
    cp, op = params_pair(s, batch=4, cc_start=1, cc_end=2)
    cp.dft_bf16 = 1
    idx = [0, 5, 10, 15]
    print(f"\n[gpu-case] dft_bf16 step n={n} K=2 B=4", flush=True)
    gc, o32, p32 = gpu_step(s, cp, idx, 1)
    oc = oracle_step(s, op, idx, 1, o32, p32)
    errs = {
        "psi_new": rel_l2(gc["psi_new"], np.stack(oc["psi_new"])),
        "factor": rel_l2(gc["factor"], np.stack(oc["factor"])),
        "n_obj": rel_l2(gc["n_obj"], oc["n_o"]),
        "n_probe": rel_l2(gc["n_probe"], oc["n_p"]),
        "O": rel_l2(gc["O"], oc["O"]),
        "P": rel_l2(gc["P"], oc["P"]),
    }
    print("dft_bf16 step relative L2 vs FP64:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < STEP_TOL, (k, v)
