"""MI355X (gfx950) block-Krylov Paraexp exp-action library (Python side).

The numerical work lives in libparaexp.so (HIP, see include/paraexp.h); this package
only binds it.  Kooij, Botchev & Geurts, arXiv 1509.04567.
"""
from .binding import (  # noqa: F401
    Context,
    PeError,
    load_library,
    LIB_PATH,
    EXPORTED,
    PE_FP64,
    PE_MIXED,
    PE_KRYLOV_POLY,
    PE_KRYLOV_SAI,
    PE_FIT_CHEBYSHEV,
    PE_FIT_SPLINE,
    PE_OK,
    PE_ERR_ARG,
    PE_ERR_NONFINITE,
    PE_ERR_DEVICE,
    PE_ERR_OOM,
    PE_ERR_UNSUPPORTED,
    FLAG_NOT_CONVERGED,
    FLAG_BREAKDOWN,
    FLAG_RANK_CAPPED,
    FLAG_FIT_CAPPED,
    workspace_query,
    policy_step,
    policy_step_growth,
    policy_reorth_skip,
    PE_STEP_ACCEPT,
    PE_STEP_REJECT,
    PE_STEP_STOP,
)
