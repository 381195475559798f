// Randomized SVD of B_k - B_0 (Alg. 3) — filled in below.
#include "common.h"

int rsvd_run(bfgsuq_ctx* h, int32_t rank, int32_t oversample, uint64_t seed, void* U, double* Sigma) {
    (void)h; (void)rank; (void)oversample; (void)seed; (void)U; (void)Sigma;
    return BFGS_ERR_STATE;
}
