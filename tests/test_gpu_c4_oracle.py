"""Every case of the 64-case batched workload against the FP64 oracle.

Case i (N in {64, 128, 192, 256}, 1-8 modes, seeds [1004, i]) is built from its
first 32 raster positions; one batch step of those 32 positions from the plain
start runs through the FP32 FFT path and through the
BF16 matrix-core DFT path, and the oracle takes the same step in FP64.  The
relative L2 errors of psi', the modulus factor, the object and probe numerators
and the updated object and probe are printed per case ("[c4-oracle]" lines) and
gated: the FP32 path at the 1e-5 parity bar (the factor at 1e-4), the BF16 path
at 1e-3 (the two-term split's bound).
"""

from __future__ import annotations

import numpy as np
import pytest

import datagen
from parity_util import gpu_step, oracle_step, params_pair, rel_l2

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP32_FACTOR_TOL = 1e-4
BF16_TOL = 1e-3
BF16_SIZES = (64, 128, 192, 256)
B = 32


def _errors(gc, oc):
    return {
        "psi_new": rel_l2(gc["psi_new"], np.stack(oc["psi_new"])),
        "factor": rel_l2(gc["factor"], np.stack(oc["factor"])),
        "n_obj": rel_l2(gc["n_obj"], oc["n_o"]),
        "n_probe": rel_l2(gc["n_probe"], oc["n_p"]),
        "O": rel_l2(gc["O"][oc["mask"]], oc["O"][oc["mask"]]),
        "P": rel_l2(gc["P"], oc["P"]),
    }


@pytest.mark.parametrize("i", range(64))
def test_c4_case_step_vs_oracle(i):
    sp = dict(datagen.random_case_spec(i))
    sp["n_pos"] = B
    s = datagen.make_scan(sp, sp["seed_key"], n_pos=B)
    n, k = s["n"], s["k"]
    print(f"\n[gpu-case] c4 case {i} N={n} K={k} B={B}", flush=True)
    cp, op = params_pair(s, batch=B, seed=1)
    idx = list(range(B))
    gc, o32, p32 = gpu_step(s, cp, idx, 1)
    oc = oracle_step(s, op, idx, 1, o32, p32)
    e32 = _errors(gc, oc)
    line = f"[c4-oracle] case {i:2d} N={n:3d} K={k} fp32 " + " ".join(f"{a}={v:.1e}" for a, v in e32.items())
    e16 = None
    if n in BF16_SIZES:
        cp.dft_bf16 = 1
        gb, _, _ = gpu_step(s, cp, idx, 1)
        e16 = _errors(gb, oc)
        line += " | bf16 " + " ".join(f"{a}={v:.1e}" for a, v in e16.items())
    print(line, flush=True)
    for a, v in e32.items():
        lim = FP32_FACTOR_TOL if a == "factor" else FP32_TOL
        assert v <= lim, f"fp32 {a}: relative L2 {v:.3e} > {lim:g}"
    if e16 is not None:
        for a, v in e16.items():
            assert v <= BF16_TOL, f"bf16 {a}: relative L2 {v:.3e} > {BF16_TOL:g}"
