/*
 * Oracle (test infrastructure only): the two-loop recursion of the paper's
 * probing algorithm (Theory & Method, "Preconditioned BFGS-based Uncertainty
 * Quantification", Alg. 2), run independently on each column of a block, in
 * plain float64 C.  It shares nothing with the GPU library.
 *
 * For a column v the recursion is
 *   q = v
 *   for i = k-1 down to 0:   r_i = 1 / (y_i^T s_i);  a_i = r_i s_i^T q;  q = q - a_i y_i
 *   z = B0 q                                         (B0 = diag(h0))
 *   for i = 0 up to k-1:     b_i = r_i y_i^T z;  z = z + s_i (a_i - b_i)
 *   optionally z = z - B0 v  (Alg. 2's last step: probe the difference B_k - B0)
 * which is the product of the inverse BFGS matrix of eq. (3) with v, built from
 * B0 by the k pairs in push order (no scaling of B0; the full-history reading).
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

/* Returns 0, or -1 if some y_i^T s_i is zero (r_i undefined). */
int oracle_two_loop(int64_t n, int32_t k, int32_t ncols, const double* h0,
                    const double* S, const double* Y, const double* V, double* out,
                    int32_t subtract_b0, int32_t nthreads) {
    double* r = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
    if (!r) return -2;
    for (int32_t i = 0; i < k; ++i) {
        double ys = dot(n, Y + (int64_t)i * n, S + (int64_t)i * n);
        if (ys == 0.0) { free(r); return -1; }
        r[i] = 1.0 / ys;
    }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int32_t j = 0; j < ncols; ++j) {
        const double* v = V + (int64_t)j * n;
        double* q = out + (int64_t)j * n;
        double* a = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
        if (!a) { bad = 1; continue; }
        for (int64_t row = 0; row < n; ++row) q[row] = v[row];
        for (int32_t i = k - 1; i >= 0; --i) {
            a[i] = r[i] * dot(n, S + (int64_t)i * n, q);
            axpy(n, -a[i], Y + (int64_t)i * n, q);
        }
        for (int64_t row = 0; row < n; ++row) q[row] *= h0[row];
        for (int32_t i = 0; i < k; ++i) {
            double b = r[i] * dot(n, Y + (int64_t)i * n, q);
            axpy(n, a[i] - b, S + (int64_t)i * n, q);
        }
        if (subtract_b0)
            for (int64_t row = 0; row < n; ++row) q[row] -= h0[row] * v[row];
        free(a);
    }
    free(r);
    return bad ? -2 : 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
