"""Pins of the scan-order generator (the "random sequence S_n" of Fig. 1, read as a
Fisher-Yates shuffle driven by SplitMix64) against the generator's published
outputs and a shuffle worked out by hand from them."""

import os

import numpy as np

import oracle as ora

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def _golden():
    vals = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                i, v = line.split()
                vals.append((int(i), int(v, 16)))
    return vals


def test_splitmix64_matches_published_outputs():
    vals = _golden()
    assert len(vals) == 3
    out = ora.splitmix64_stream(0, len(vals))
    for i, v in vals:
        assert out[i] == v, f"output {i}: {out[i]:016x} != {v:016x}"


def test_permutation_worked_by_hand():
    # seed 1, iteration 1 -> generator state 1 XOR 1 = 0, so the draws are the
    # published outputs above.  n = 3: i = 2 takes j = 0xe220a8397b1dcdaf mod 3;
    # 16 = 1 (mod 3), so this is the sum of the hex digits (130) mod 3 = 1: swap
    # a[2] and a[1] -> [0, 2, 1].  i = 1 takes j = 0x6e789e6aa1b965f4 mod 2 = 0
    # (even): swap a[1] and a[0] -> [2, 0, 1].
    assert ora.permutation(1, 1, 3).tolist() == [2, 0, 1]
    # n = 2 uses only the first draw: j = 0xe220a8397b1dcdaf mod 2 = 1 (odd): no change
    assert ora.permutation(1, 1, 2).tolist() == [0, 1]


def test_permutation_is_uniform_over_small_n():
    # a Fisher-Yates shuffle driven by a good generator hits each of the 3! orders
    # about equally often; a wrong index range (e.g. j = next mod i) cannot produce
    # the identity and would fail this
    counts = {}
    for t in range(1, 6001):
        key = tuple(ora.permutation(12345, t, 3).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    assert all(abs(c - 1000) < 150 for c in counts.values()), counts
