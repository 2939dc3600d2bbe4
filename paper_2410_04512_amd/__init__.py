"""Support-graph preconditioned CG for cell-based models on MI355X.

The compute path is the HIP library libsgp.so (C ABI in include/sgp.h); this
package only marshals arguments to it (see sgp.py).  There is no fallback:
without the built library every call raises.
"""
from .sgp import (  # noqa: F401
    SgpError, Context, Graph, Bsr, Tree, Prec, Mpnn, Step, lib, LIB_PATH,
    SCHED_LEVEL, SCHED_CONTRACT, OK, EINVAL, ENOMEM, EHIP, ECAPACITY, ENOTSPD, ENOCONV,
    EBREAKDOWN, ENONFINITE, ESTALE,
)
