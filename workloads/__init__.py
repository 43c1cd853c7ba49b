"""Seeded synthetic inputs for tensor robust PCA.

This package only draws random tensors (a low-rank Tucker part plus a sparse
corruption) with the shapes and value distributions of the paper's synthetic
workloads (Section 5.1) and of the configurations benchmarked here.  It holds
none of the solver's arithmetic, so both the FP64 oracle and the GPU path can
take their inputs from it without sharing any solver code.
"""

from .generators import (  # noqa: F401
    CONFIGS,
    Workload,
    haar_stiefel,
    make_config,
    materialise,
    mri_standin,
    psnr,
    serving_trace,
    tucker,
    tucker_workload,
    video_workload,
)
