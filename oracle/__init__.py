"""FP64 CPU oracle for partially coherent ptychography (pc-ePIE).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the GPU library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the HIP library and its Python binding) never does, and shares no code,
tables or constants with it.

Every function cites the passage of the paper (Xu et al., "A high-performance
reconstruction method for partially coherent ptychography", arXiv 2406.06640)
it follows.  Where the paper is silent the reading used is stated in the
docstring; the same readings are listed in the design notes of the repository.

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` except the mini-batch generalisation of the ePIE
update for batch size B > 1, which the paper does not define (it is pinned only
by its B = 1 reduction to sequential ePIE and by convergence): parity unpinned
for B > 1 beyond those properties.

``oracle.pcdm`` is the FP64 pc-DM engine (the difference map with boxes 1 and
2, Sec. 4.5), pinned by the least-squares property of its overlap projection,
the consistent-data fixed point, the single-position reduction to the Fourier
modulus projection and noise-free convergence (``tests/test_oracle_dm.py``).

``oracle.pclsqml`` is the FP64 pc-LSQML engine (LSQML of ref. [27] with boxes 1
and 2, Sec. 3.2 and 4.1), pinned by library least squares on its step pair
(undamped and damped), the consistent-data fixed point, the single-position
landing on the modulus projection, the closed-form steps of one position and
noise-free convergence (``tests/test_oracle_lsqml.py``).
"""

from .pcepie import *  # noqa: F401,F403
