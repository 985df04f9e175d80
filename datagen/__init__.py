"""Seeded synthetic ptychography scans (shared input generator).

This package simulates measurements only: object and probe textures, scan
positions, and recorded intensities from the coherent forward model (Eq. 1)
blurred by the partial-coherence model (Eq. 2), plus Poisson counting noise.
It holds none of the reconstruction's arithmetic and is the only code that
both the oracle's tests and the GPU library's tests and benchmark share.
"""

from .synth import *  # noqa: F401,F403
