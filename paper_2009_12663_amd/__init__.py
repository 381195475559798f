"""MI355X-native BFGS inverse Hessian, randomized SVD and posterior variance.

The computation lives in libbfgsuq.so (HIP, gfx950); this package is its thin
Python binding.  See include/bfgsuq.h for the C ABI.
"""
from ._lib import (  # noqa: F401
    Bfgs,
    BfgsBatch,
    Mlp,
    BfgsError,
    bfgs_create,
    bfgs_push_pair,
    bfgs_apply_Hinv,
    bfgs_apply_Hdiff,
    bfgs_rsvd,
    bfgs_posterior_diag,
    bfgs_generate_probes,
    bfgs_destroy,
    load,
    LIB_PATH,
    EXPORTS,
    BFGS_OK,
    BFGS_ERR_ARG,
    BFGS_ERR_FULL,
    BFGS_ERR_STATE,
    BFGS_ERR_CURVATURE,
    BFGS_ERR_NONFINITE,
    BFGS_ERR_NUMERIC,
    tsqr_shape,
    precond_diag,
    GridOp,
    minimize_quadratic,
)
