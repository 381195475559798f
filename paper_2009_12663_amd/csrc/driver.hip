// Full-history BFGS on a quadratic, resident on the GPU (Alg. 1 with every pair
// kept and B_0 fixed, the search direction of eq. (1)), and the synthetic Hessian
// it runs on.
//
// The paper obtains its pairs from elastic FWI; here the misfit is the quadratic
// 1/2 m^T A m - b^T m whose Hessian A stands in for the wave-equation Hessian:
//   A = diag(D) + P (x) (G_z (x) G_x),   P = I + c (1 1^T - I) over the parameter fields,
// with G_x, G_z the truncated Gaussian smoothers (weights exp(-t^2 / (2 sigma^2)),
// |t| <= half, normalised to sum 1, zero outside the grid), applied by a stencil.
//
// One iteration:  p = -B_k g (bfgs_apply_Hinv with one column; p = -g before the
// first pair when B_0 = gamma I), the exact line search alpha = -g^T p / p^T A p,
// s = alpha p, y = A s = alpha A p (formed from A p, not by differencing
// gradients), m += s, g += y, then (s, y) is pushed.  Dot products are fixed-order
// block reductions in float64, so a run is deterministic.
#include <cmath>
#include <new>
#include <vector>

#include "common.h"

struct bfgsuq_gridop {
    int64_t nx = 0, nz = 0, n = 0;
    int32_t nparam = 0, half = 0;
    double coupling = 0.0;
    hipStream_t stream = nullptr;
    double* D = nullptr;       // n
    double* w = nullptr;       // 2 half + 1 normalised weights
    double* tmp = nullptr;     // 2 n (x pass, z pass)
};

namespace {

constexpr int kRedBlocks = 256;

int blocks_for(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

__global__ void stencil_x(int64_t nx, int64_t rows, int half, const double* __restrict__ w, const double* __restrict__ x,
                          double* __restrict__ out) {
    const int64_t total = rows * nx;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = e % nx;
        const double* src = x + (e - ix);
        double s = 0.0;
        const int lo = (int)max((int64_t)-half, -ix), hi = (int)min((int64_t)half, nx - 1 - ix);
        for (int t = lo; t <= hi; ++t) s = fma(w[t + half], src[ix + t], s);
        out[e] = s;
    }
}

__global__ void stencil_z(int64_t nx, int64_t nz, int64_t nparam, int half, const double* __restrict__ w,
                          const double* __restrict__ x, double* __restrict__ out) {
    const int64_t total = nparam * nz * nx;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = e % nx, iz = (e / nx) % nz, p = e / (nx * nz);
        const double* src = x + p * nz * nx + ix;
        double s = 0.0;
        const int lo = (int)max((int64_t)-half, -iz), hi = (int)min((int64_t)half, nz - 1 - iz);
        for (int u = lo; u <= hi; ++u) s = fma(w[u + half], src[(iz + u) * nx], s);
        out[e] = s;
    }
}

// y = D o x + (1 - c) g + c sum_q g_q, g the smoothed fields (coupling P applied per point).
__global__ void couple(int64_t npt, int nparam, double c, const double* __restrict__ D, const double* __restrict__ x,
                       const double* __restrict__ g, double* __restrict__ y) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npt; e += (int64_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        for (int p = 0; p < nparam; ++p) sum += g[(int64_t)p * npt + e];
        for (int p = 0; p < nparam; ++p) {
            const int64_t i = (int64_t)p * npt + e;
            y[i] = fma(D[i], x[i], fma(1.0 - c, g[i], c * sum));
        }
    }
}

// Fixed-order dot products: per-block partials, then one block sums them in order.
__global__ void dot_partial(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        s = fma(a[e], b[e], s);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void dot_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// alpha = -(g^T p) / (p^T A p) from the two dots in sc[0], sc[1]; s = alpha p, y = alpha A p,
// m += s, g += y.
__global__ void line_step(int64_t n, const double* __restrict__ sc, const double* __restrict__ p,
                          const double* __restrict__ Ap, double* __restrict__ s, double* __restrict__ y,
                          double* __restrict__ m, double* __restrict__ g, double damping) {
    const double alpha = damping * (-sc[0] / sc[1]);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double se = alpha * p[e], ye = alpha * Ap[e];
        s[e] = se;
        y[e] = ye;
        m[e] += se;
        g[e] += ye;
    }
}

__global__ void negate_to(int64_t n, const double* __restrict__ x, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = -x[e];
}

template <typename Ti, typename To>
__global__ void convert(int64_t n, const Ti* __restrict__ x, To* __restrict__ out, double scale) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (To)(scale * (double)x[e]);
}

int gridop_apply_impl(bfgsuq_gridop* op, const double* x, double* y, hipStream_t st) {
    const int64_t n = op->n;
    double* tx = op->tmp;
    double* tz = op->tmp + n;
    hipLaunchKernelGGL(stencil_x, dim3(blocks_for(n)), dim3(256), 0, st, op->nx, op->nz * (int64_t)op->nparam, op->half,
                       op->w, x, tx);
    hipLaunchKernelGGL(stencil_z, dim3(blocks_for(n)), dim3(256), 0, st, op->nx, op->nz, (int64_t)op->nparam, op->half,
                       op->w, tx, tz);
    const int64_t npt = op->nx * op->nz;
    hipLaunchKernelGGL(couple, dim3(blocks_for(npt)), dim3(256), 0, st, npt, op->nparam, op->coupling, op->D, x, tz, y);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

void launch_dot(int64_t n, const double* a, const double* b, double* part, double* out, hipStream_t st) {
    hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(256), 0, st, n, a, b, part);
    hipLaunchKernelGGL(dot_final, dim3(1), dim3(256), 0, st, kRedBlocks, part, out);
}

}  // namespace

extern "C" {

int bfgs_gridop_destroy(bfgs_gridop_t op) {
    if (!op) return BFGS_OK;
    (void)hipStreamSynchronize(op->stream);
    if (op->D) (void)hipFree(op->D);
    if (op->w) (void)hipFree(op->w);
    if (op->tmp) (void)hipFree(op->tmp);
    delete op;
    return BFGS_OK;
}

int bfgs_gridop_create(int64_t nx, int64_t nz, int32_t nparam, const double* D, double sigma, int32_t half,
                       double coupling, void* stream, bfgs_gridop_t* out) {
    if (!out || !D || nx < 1 || nz < 1 || nparam < 1 || !(sigma > 0.0) || !std::isfinite(sigma) || half < 0 ||
        half > 4096 || !std::isfinite(coupling))
        return BFGS_ERR_ARG;
    *out = nullptr;
    bfgsuq_gridop* op = new (std::nothrow) bfgsuq_gridop();
    if (!op) return BFGS_ERR_ALLOC;
    op->nx = nx;
    op->nz = nz;
    op->nparam = nparam;
    op->n = nx * nz * (int64_t)nparam;
    op->half = half;
    op->coupling = coupling;
    op->stream = (hipStream_t)stream;
    std::vector<double> w(2 * half + 1);
    double sum = 0.0;
    for (int t = -half; t <= half; ++t) sum += (w[t + half] = std::exp(-0.5 * (t / sigma) * (t / sigma)));
    for (double& v : w) v /= sum;
    if (hipMalloc(&op->D, op->n * 8) != hipSuccess || hipMalloc(&op->w, w.size() * 8) != hipSuccess ||
        hipMalloc(&op->tmp, 2 * op->n * 8) != hipSuccess) {
        bfgs_gridop_destroy(op);
        return BFGS_ERR_ALLOC;
    }
    if (hipMemcpyAsync(op->D, D, op->n * 8, hipMemcpyDeviceToDevice, op->stream) != hipSuccess ||
        hipMemcpyAsync(op->w, w.data(), w.size() * 8, hipMemcpyHostToDevice, op->stream) != hipSuccess ||
        hipStreamSynchronize(op->stream) != hipSuccess) {
        bfgs_gridop_destroy(op);
        return BFGS_ERR_HIP;
    }
    *out = op;
    return BFGS_OK;
}

int bfgs_gridop_apply(bfgs_gridop_t op, const double* x, int32_t ncols, double* y) {
    if (!op || !x || !y || ncols < 1 || x == y) return BFGS_ERR_ARG;
    for (int j = 0; j < ncols; ++j) {
        const int rc = gridop_apply_impl(op, x + (int64_t)j * op->n, y + (int64_t)j * op->n, op->stream);
        if (rc != BFGS_OK) return rc;
    }
    return BFGS_OK;
}

int bfgs_minimize_quadratic(bfgs_t h, bfgs_gridop_t op, const double* b, int32_t max_iter, double rel_tol, double* m,
                            double* gnorm, int32_t* iters) {
    return bfgs_minimize_quadratic_ex(h, op, b, max_iter, rel_tol, 0, 1.0, m, gnorm, iters);
}

int bfgs_minimize_quadratic_ex(bfgs_t h, bfgs_gridop_t op, const double* b, int32_t max_iter, double rel_tol,
                               int32_t memory, double damping, double* m, double* gnorm, int32_t* iters) {
    if (!h || !op || !b || !m || !iters || max_iter < 0 || !(rel_tol >= 0.0) || op->n != h->n) return BFGS_ERR_ARG;
    if (memory < 0 || memory > h->kmax || !(damping > 0.0 && damping <= 1.0)) return BFGS_ERR_ARG;
    if (memory > 0 && h->streamed) return BFGS_ERR_STATE;   // the window moves in device memory
    if (h->storage == BFGS_BF16) return BFGS_ERR_ARG;   // a bfloat16 gradient cannot reach small tolerances
    if (h->k != 0) return BFGS_ERR_STATE;                // the run starts from m = 0 with an empty history
    if (op->stream != h->stream) return BFGS_ERR_ARG;
    *iters = 0;
    const int64_t n = h->n;
    hipStream_t st = h->stream;
    const bool f32 = h->storage == BFGS_F32;
    // g, p, Ap, s, y (float64), the float32 copies of g and p, partial sums and scalars
    void* ws = nullptr;
    const size_t bytes = (size_t)5 * n * 8 + (f32 ? 2 * (size_t)n * 4 : 0) + (kRedBlocks + 8) * 8;
    if (hipMalloc(&ws, bytes) != hipSuccess) return BFGS_ERR_ALLOC;
    double* g = (double*)ws;
    double* p = g + n;
    double* Ap = p + n;
    double* s = Ap + n;
    double* y = s + n;
    float* g32 = f32 ? (float*)(y + n) : nullptr;
    float* p32 = f32 ? g32 + n : nullptr;
    double* part = f32 ? (double*)(p32 + n) : y + n;
    double* sc = part + kRedBlocks;   // [0] g^T p, [1] p^T A p, [2] g^T g
    int rc = BFGS_OK;
    double host[3];
    auto gg = [&](double* out) -> int {
        launch_dot(n, g, g, part, sc + 2, st);
        if (hipMemcpyAsync(host + 2, sc + 2, 8, hipMemcpyDeviceToHost, st) != hipSuccess) return BFGS_ERR_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return BFGS_ERR_HIP;
        *out = std::sqrt(host[2]);
        return std::isfinite(*out) ? BFGS_OK : BFGS_ERR_NONFINITE;
    };
    hipLaunchKernelGGL(negate_to, dim3(blocks_for(n)), dim3(256), 0, st, n, b, g);   // g_0 = A 0 - b
    if (hipMemsetAsync(m, 0, n * 8, st) != hipSuccess) rc = BFGS_ERR_HIP;
    double gn0 = 0.0;
    if (rc == BFGS_OK) rc = gg(&gn0);
    if (rc == BFGS_OK && gnorm) gnorm[0] = gn0;
    int it = 0;
    while (rc == BFGS_OK && it < max_iter && (memory > 0 || h->k < h->kmax)) {
        if (h->k == 0 && h->gamma_mode) {
            hipLaunchKernelGGL(negate_to, dim3(blocks_for(n)), dim3(256), 0, st, n, g, p);   // gamma unknown: p = -g
        } else if (f32) {
            hipLaunchKernelGGL((convert<double, float>), dim3(blocks_for(n)), dim3(256), 0, st, n, g, g32, 1.0);
            if ((rc = apply_block(h, g32, 1, p32, false)) != BFGS_OK) break;
            hipLaunchKernelGGL((convert<float, double>), dim3(blocks_for(n)), dim3(256), 0, st, n, p32, p, -1.0);
        } else {
            if ((rc = apply_block(h, g, 1, p, false)) != BFGS_OK) break;
            hipLaunchKernelGGL(negate_to, dim3(blocks_for(n)), dim3(256), 0, st, n, p, p);
        }
        if ((rc = gridop_apply_impl(op, p, Ap, st)) != BFGS_OK) break;
        launch_dot(n, g, p, part, sc + 0, st);
        launch_dot(n, p, Ap, part, sc + 1, st);
        hipLaunchKernelGGL(line_step, dim3(blocks_for(n)), dim3(256), 0, st, n, sc, p, Ap, s, y, m, g, damping);
        if (hipGetLastError() != hipSuccess) {
            rc = BFGS_ERR_HIP;
            break;
        }
        // the limited-memory form keeps the last `memory` pairs
        if (memory > 0 && h->k == memory && (rc = pop_oldest(h)) != BFGS_OK) break;
        if ((rc = bfgs_push_pair(h, s, y, BFGS_F64)) != BFGS_OK) break;
        ++it;
        double gn = 0.0;
        if ((rc = gg(&gn)) != BFGS_OK) break;
        if (gnorm) gnorm[it] = gn;
        if (gn <= rel_tol * gn0) break;
    }
    *iters = it;
    (void)hipStreamSynchronize(st);
    (void)hipFree(ws);
    return rc;
}

}  // extern "C"
