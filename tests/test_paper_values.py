"""The paper-scan workload of bench.py against the values the paper prints
(tests/golden/paper_qpt_scans.txt, each line citing its table or caption)."""

from __future__ import annotations

import math
import os

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_qpt_scans.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, value = line.split()[:2]
                vals[key] = float(value)
    return vals


def test_paper_scan_shapes_follow_table_1():
    g = _golden()
    shapes = {name: (geom, step, fpx, ms) for name, geom, step, fpx, ms in bench.PAPER_SHAPES}
    assert bench.PAPER_FRAME == g["pattern_size_px"]
    assert bench.PAPER_SCAN_SIDE ** 2 == g["scan_points"]
    step_um = g["scan_step_mm"] * 1000.0
    # scan step in object pixels, rounded to the nearest whole pixel
    assert shapes["far"][1] == round(step_um / g["object_pixel_far_um"])
    assert shapes["near"][1] == round(step_um / g["object_pixel_near_um"])
    # Fresnel number per pixel of the near-field geometry: dx^2 / (lambda z)
    f_px = g["detector_pixel_um"] ** 2 / (g["near_wavelength_nm"] * 1e-3 * g["near_distance_mm"] * 1e3)
    assert math.isclose(shapes["near"][2], f_px, rel_tol=2e-3)
    assert shapes["far"][2] == 0.0
    assert shapes["far"][3] == g["pcepie_ms_per_iteration_far"]
    assert shapes["near"][3] == g["pcepie_ms_per_iteration_near"]


def test_default_kernel_size_is_the_papers():
    import paper_2406_06640_amd as P
    assert P.default_params().kernel_size == _golden()["kernel_size_px"]
