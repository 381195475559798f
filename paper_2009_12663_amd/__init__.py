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
)
