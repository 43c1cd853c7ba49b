"""MI355X (gfx950) PASD solver for tensor robust PCA.

The solver is the HIP library libpasd.so behind the C ABI in include/pasd.h;
this package holds its sources (csrc/), its build step (build.py) and a thin
ctypes binding (pasd.py).
"""

from .pasd import (  # noqa: F401
    BF16_GEMM, FP32, FP64, PasdError, Q_D, Q_E, Q_P, Q_SCALARS, Q_U, Q_UF, Q_WEV, Q_X, Q_Y, Q_Z,
    Solver,
    footprint, lib, make_config, step_batch, validate)
