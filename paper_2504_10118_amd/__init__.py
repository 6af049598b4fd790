"""MI355X (gfx950) MAGPIE ptychography hot path: HIP kernels behind a C ABI.

The solver (arXiv 2504.10118, Alg 3 and Alg 4 with minibatches) runs in
``lib/libmagpie.so``, built from ``csrc/`` by ``python -m
paper_2504_10118_amd.build``.  This package only marshals arguments.
"""

from .magpie import (  # noqa: F401
    C64,
    C128,
    CNN,
    COARSE_C64,
    COARSE_C128,
    COARSE_LOGPOLAR,
    W_BF16,
    W_F32,
    UPDATE_PROBE,
    PHASE_RECYCLE,
    PROBE_ALTERNATE,
    PERSISTENT,
    GRAPH,
    LIB_PATH,
    Magpie,
    MagpieError,
    list_plans,
    load_library,
    permutation,
    restrict_object,
    run_epochs_multi,
)
