"""FP64 CPU oracle for MAGPIE (arXiv 2504.10118) -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy implementation of what the GPU hot
path computes, written from the paper.  It exists to check the HIP kernels:
only the test suite, the smoke check of the entry module and the CPU-baseline
leg of the benchmark may import it.  The product path never calls it and
shares no code with it (the two meet only in the seeded generators of
``synth/``, which hold none of the method's arithmetic).

Every function cites the passage of the paper it follows.  All arithmetic is
complex128 / float64.  Readings of points the paper leaves open are stated
where they are used.

Parity status of each part is in the module docstring of ``oracle.core``.
"""

from .core import *  # noqa: F401,F403
from . import learned  # noqa: F401
