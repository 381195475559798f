/*
 * Oracle (test infrastructure only): the inverse BFGS matrix of eq. (3), built
 * from B_0 = diag(h0) by the stored pairs in push order, applied to a block of
 * vectors, in plain float64 C.  It shares nothing with the GPU library.
 *
 * Eq. (3) takes B_i to B_{i+1} with the pair (s_i, y_i) and r_i = 1 / (y_i^T s_i):
 *     B_{i+1} = (I - r_i s_i y_i^T) B_i (I - r_i y_i s_i^T) + r_i s_i s_i^T.
 * Multiplying out for one vector v, with t = s_i^T v,
 *     B_{i+1} v = (I - r_i s_i y_i^T) [ B_i (v - r_i t y_i) ] + r_i t s_i,
 * i.e. one application of B_i to w = v - r_i t y_i, after which z = B_i w is
 * corrected by z + r_i (t - y_i^T z) s_i.  apply_level() is that identity as a
 * recursion on i, bottoming out at B_0 v = h0 o v; nothing is reordered or
 * fused.  With `subtract_b0` the result is (B_k - B_0) v, the operator the
 * randomized SVD (Alg. 3) samples.
 *
 * Layout: S, Y, V, out are column-major with leading dimension n (column i of S
 * is s_i, contiguous).  Columns are independent; OpenMP runs them in parallel.
 */
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

static double dot(int64_t n, const double* a, const double* b) {
    double acc = 0.0;
    for (int64_t r = 0; r < n; ++r) acc += a[r] * b[r];
    return acc;
}

static void axpy(int64_t n, double alpha, const double* x, double* y) {
    for (int64_t r = 0; r < n; ++r) y[r] += alpha * x[r];
}

/* v <- B_level v, in place (level pairs: s_0 .. s_{level-1}). */
static void apply_level(int32_t level, int64_t n, const double* h0, const double* S, const double* Y,
                        const double* rinv, double* v) {
    if (level == 0) {
        for (int64_t row = 0; row < n; ++row) v[row] *= h0[row];
        return;
    }
    const int32_t i = level - 1;
    const double* s = S + (int64_t)i * n;
    const double* y = Y + (int64_t)i * n;
    const double t = dot(n, s, v);
    axpy(n, -rinv[i] * t, y, v);                 /* w = v - r t y            */
    apply_level(i, n, h0, S, Y, rinv, v);        /* z = B_i w                */
    const double u = dot(n, y, v);
    axpy(n, rinv[i] * (t - u), s, v);            /* z + r (t - y^T z) s      */
}

/* Returns 0, or -1 if some y_i^T s_i is zero (r_i undefined). */
int oracle_apply_hk(int64_t n, int32_t k, int32_t ncols, const double* h0, const double* S, const double* Y,
                    const double* V, double* out, int32_t subtract_b0, int32_t nthreads) {
    double* rinv = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
    if (!rinv) return -2;
    for (int32_t i = 0; i < k; ++i) {
        const double ys = dot(n, Y + (int64_t)i * n, S + (int64_t)i * n);
        if (ys == 0.0) { free(rinv); return -1; }
        rinv[i] = 1.0 / ys;
    }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int32_t j = 0; j < ncols; ++j) {
        const double* v = V + (int64_t)j * n;
        double* z = out + (int64_t)j * n;
        for (int64_t row = 0; row < n; ++row) z[row] = v[row];
        apply_level(k, n, h0, S, Y, rinv, z);
        if (subtract_b0)
            for (int64_t row = 0; row < n; ++row) z[row] -= h0[row] * v[row];
    }
    free(rinv);
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
