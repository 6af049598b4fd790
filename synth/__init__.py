"""Seeded synthetic inputs for MAGPIE ptychography runs.

This module is shared by the FP64 oracle (``oracle/``) and by the GPU path
(``paper_2504_10118_amd``).  It holds none of the method's arithmetic: no
Fourier transform, no revised exit wave, no surrogate step.  It only draws
the things a ptychography experiment is made of -- an object, a probe, a
jittered raster scan, Poisson counts for given noiseless intensities, and
epoch permutations -- from numpy PCG64 streams.

The paper's own inputs (a zone-plate probe, two 512x512 image objects;
Section 5, "Probe" and "Object" paragraphs) are not available, so these
generators stand in for them with the shapes, overlap and photon levels of
the paper's workloads (Section 5 setup; Poisson model of the "Noise level"
paragraph, re-parameterised by peak photon count).
"""

from .generators import (  # noqa: F401
    WORKLOADS,
    ScanConfig,
    workload_rngs,
    make_object,
    make_probe,
    make_scan,
    poisson_counts,
    poisson_counts_device,
    epoch_orders,
    make_problem_inputs,
    BatchedRecon,
    batched_workload,
    make_batched_inputs,
    make_objects_device,
)
