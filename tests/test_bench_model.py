"""Host-side accounting of bench.py (no GPU): the per-slot byte model behind the
dominant kernel's roofline, the rule for the paired inverse row pass, and the
method-level pass model behind the graded fraction, each against closed forms
worked out by hand for small cases."""

from __future__ import annotations

import math

import bench


def test_paired_rows_rule():
    # power-of-two frames up to 512 with at least two slots per batch
    for n in (8, 16, 32, 64, 128, 256, 512):
        assert bench.paired_rows(n, 2) and bench.paired_rows(n, 32)
        assert not bench.paired_rows(n, 1)
    for n in (24, 48, 96, 192, 384, 768, 1024):
        assert not bench.paired_rows(n, 32)


def test_per_slot_bytes_closed_forms():
    n, k = 256, 4
    nn = n * n
    # inverse row pass: K frames in (8K), probe contributions out (8K, or 4K per slot when
    # two slots share one frame set), box in (8) and object numerator out (8)
    assert bench.per_slot_bytes("inv_rows_update", n, k) == (8 * k + 8 * k + 16) * nn
    assert bench.per_slot_bytes("inv_rows_update", n, k, pairs=True) == (8 * k + 4 * k + 16) * nn
    # the update reads what the row pass wrote
    assert bench.per_slot_bytes("obj_probe_update", n, k) == (8 * k + 12) * nn
    assert bench.per_slot_bytes("obj_probe_update", n, k, pairs=True) == (4 * k + 12) * nn
    # pairing changes nothing upstream of the inverse row pass
    for name in ("fwd_rows", "fwd_cols", "modulus_factor", "inv_cols"):
        assert bench.per_slot_bytes(name, n, k) == bench.per_slot_bytes(name, n, k, pairs=True)
    # near field: the forward column pass writes its frames back
    assert bench.per_slot_bytes("fwd_cols", n, k, near=True) == (16 * k + 4) * nn
    # a 134 217 728-byte launch: 32 slots of the paired pass at 256^2, K = 4
    assert 32 * bench.per_slot_bytes("inv_rows_update", n, k, pairs=True) == 134217728
    assert bench.per_slot_bytes("no_such_kernel", n, k) is None


def test_pass_model_two_disjoint_boxes():
    n, k = 16, 2
    nn = n * n
    positions = [(0, 0), (100, 100)]  # boxes that do not overlap
    m = bench.pass_model(n, k, False, positions, [0, 1], 2)
    # flop: K n_fft 5 N^2 log2(N^2) + (30K + 60) N^2 per position, n_fft = 2 in the far field
    flop = 2 * (k * 2 * 5 * nn * 2 * math.log2(n) + (30 * k + 60) * nn)
    assert m["flop"] == flop
    # bytes: 12 N^2 per position, one batch: 16 |union| (two whole boxes) + 16 K N^2
    b_min = 12 * nn * 2 + 16 * (2 * nn) + 16 * k * nn
    assert m["bytes_min"] == b_min
    assert m["bytes_pass"] == b_min + 32 * k * nn * 2


def test_pass_model_union_counts_overlap_once():
    n, k = 8, 1
    nn = n * n
    # two boxes shifted by 4 columns: the union is 8 rows x 12 columns
    m = bench.pass_model(n, k, False, [(0, 0), (0, 4)], [0, 1], 2)
    assert m["bytes_min"] == 12 * nn * 2 + 16 * (8 * 12) + 16 * k * nn
    # in separate batches each box is read and written on its own
    m1 = bench.pass_model(n, k, False, [(0, 0), (0, 4)], [0, 1], 1)
    assert m1["bytes_min"] == 12 * nn * 2 + 2 * (16 * nn + 16 * k * nn)
    # near field: four transforms per direction and (42K + 60) N^2 element-wise flop
    mn = bench.pass_model(n, k, True, [(0, 0)], [0], 1)
    assert mn["flop"] == k * 4 * 5 * nn * 2 * math.log2(n) + (42 * k + 60) * nn
