"""FP64 CPU oracle for the PASD ADMM (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it, and it shares no code
with the GPU library: both take their inputs from the ``workloads`` package.
"""

from .pasd_oracle import (  # noqa: F401
    OracleState,
    default_lambdas,
    fold,
    pasd_init,
    pasd_iterate,
    pasd_output,
    pasd_solve,
    polar,
    procrustes_keep,
    prox_l1,
    svt,
    unfold,
)
from .horpca_oracle import horpca_admm  # noqa: F401
