// The diagonal initial inverse Hessian of eq. (4), B_0 = (H_0 + lambda I)^-1, from a
// per-point diagonal Hessian estimate H_0 (the role diag(J^T J) plays in the
// paper's preconditioners P1-P4), smoothed and damped as the paper prescribes for
// all four of them: the estimate is smoothed per parameter field the way a gradient
// is smoothed (a separable Gaussian here), and the inverse is stabilised with the
// median of the smoothed estimate, lambda = damping * median.
//
//   smooth   hs(p, iz, ix) = sum_{t,u} w_t w_u h(p, iz + u, ix + t) / (sum_t w_t)(sum_u w_u),
//            the sums over the taps that fall inside the grid (a constant field stays
//            constant up to the edges), w_t = exp(-t^2 / (2 sigma^2)), |t| <= half;
//            the x pass then the z pass, float64 sums, hs rounded to float32
//   median   the two middle order statistics of hs (float32) by a radix select on
//            the bit patterns (positive floats order as unsigned integers),
//            averaged in float64 (the mean of the two middle values for even n)
//   h0       1 / (hs + lambda), float64, rounded to float32
#include <cmath>
#include <vector>

#include "common.h"

namespace {

constexpr int kMaxHalf = 512;

__global__ void smooth_x(int64_t nx, int64_t rows, int half, const double* __restrict__ w, const float* __restrict__ h,
                         double* __restrict__ out) {
    const int64_t total = rows * nx;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = e % nx, row = e / nx;
        const float* src = h + row * nx;
        double s = 0.0, wn = 0.0;
        for (int t = -half; t <= half; ++t) {
            const int64_t j = ix + t;
            if (j < 0 || j >= nx) continue;
            s = fma(w[t + half], (double)src[j], s);
            wn += w[t + half];
        }
        out[e] = s / wn;
    }
}

// z pass over the x-smoothed field (float64), rounding the result to float32.
__global__ void smooth_z(int64_t nx, int64_t nz, int64_t nparam, int half, const double* __restrict__ w,
                         const double* __restrict__ hx, float* __restrict__ hs) {
    const int64_t total = nparam * nz * nx;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = e % nx, iz = (e / nx) % nz, p = e / (nx * nz);
        const double* src = hx + p * nz * nx + ix;
        double s = 0.0, wn = 0.0;
        for (int u = -half; u <= half; ++u) {
            const int64_t j = iz + u;
            if (j < 0 || j >= nz) continue;
            s = fma(w[u + half], src[j * nx], s);
            wn += w[u + half];
        }
        hs[e] = (float)(s / wn);
    }
}

// Radix select state of one order statistic: the key's bits found so far (prefix,
// under mask) and the rank still sought among the keys that share them.
struct SelectState {
    uint32_t prefix, mask, rank, pad;
};

__global__ void select_init(SelectState* st, uint32_t r0, uint32_t r1, uint32_t* hist) {
    if (threadIdx.x < 2) {
        st[threadIdx.x].prefix = 0u;
        st[threadIdx.x].mask = 0u;
        st[threadIdx.x].rank = threadIdx.x == 0 ? r0 : r1;
        st[threadIdx.x].pad = 0u;
    }
    for (int i = threadIdx.x; i < 512; i += blockDim.x) hist[i] = 0u;
}

// Histogram of the 8 bits at `shift` of the keys that share each state's prefix.
__global__ void select_hist(int64_t n, const float* __restrict__ x, const SelectState* __restrict__ st, int shift,
                            uint32_t* __restrict__ hist) {
    __shared__ uint32_t local[512];
    for (int i = threadIdx.x; i < 512; i += blockDim.x) local[i] = 0u;
    __syncthreads();
    const SelectState s0 = st[0], s1 = st[1];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = __float_as_uint(x[e]);
        const uint32_t bin = (key >> shift) & 255u;
        if ((key & s0.mask) == s0.prefix) atomicAdd(&local[bin], 1u);
        if ((key & s1.mask) == s1.prefix) atomicAdd(&local[256 + bin], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 512; i += blockDim.x)
        if (local[i]) atomicAdd(&hist[i], local[i]);
}

// One thread per state: the bin that holds the sought rank; the histogram is cleared
// for the next pass.
__global__ void select_pick(SelectState* st, int shift, uint32_t* hist) {
    __shared__ uint32_t h[512];
    for (int i = threadIdx.x; i < 512; i += blockDim.x) h[i] = hist[i];
    __syncthreads();
    for (int i = threadIdx.x; i < 512; i += blockDim.x) hist[i] = 0u;
    if (threadIdx.x < 2) {
        SelectState s = st[threadIdx.x];
        const uint32_t* hh = h + 256 * threadIdx.x;
        uint32_t below = 0u;
        int b = 0;
        for (; b < 255; ++b) {
            if (below + hh[b] > s.rank) break;
            below += hh[b];
        }
        s.rank -= below;
        s.prefix |= (uint32_t)b << shift;
        s.mask |= 255u << shift;
        st[threadIdx.x] = s;
    }
}

__global__ void precond_finish(int64_t n, const float* __restrict__ hs, const SelectState* __restrict__ st,
                               double damping, float* __restrict__ h0, double* __restrict__ lambda_out) {
    const double lo = (double)__uint_as_float(st[0].prefix), hi = (double)__uint_as_float(st[1].prefix);
    const double lam = damping * (0.5 * (lo + hi));
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        h0[e] = (float)(1.0 / ((double)hs[e] + lam));
    if (blockIdx.x == 0 && threadIdx.x == 0) lambda_out[0] = lam;
}

int grid_blocks(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (int)(g > 2048 ? 2048 : (g < 1 ? 1 : g));
}

}  // namespace

extern "C" int bfgs_precond_diag(int64_t nx, int64_t nz, int32_t nparam, const float* hdiag, double sigma,
                                 int32_t half, double damping, float* h0_out, float* hs_out, double* lambda_out,
                                 void* stream) {
    if (nx < 1 || nz < 1 || nparam < 1 || !hdiag || !h0_out || !(sigma > 0.0) || half < 0 || half > kMaxHalf ||
        !(damping >= 0.0) || !std::isfinite(sigma) || !std::isfinite(damping))
        return BFGS_ERR_ARG;
    const int64_t n = nx * nz * (int64_t)nparam;
    if (n > (int64_t)0xFFFFFFFFll) return BFGS_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> w(2 * half + 1);
    for (int t = -half; t <= half; ++t) w[t + half] = std::exp(-0.5 * (t / sigma) * (t / sigma));
    // scratch: taps | x-smoothed field (float64) | smoothed field (float32) | select state | histograms | lambda
    const size_t off_hx = 8 * (size_t)(2 * kMaxHalf + 1 + 7) / 8 * 8;
    const size_t off_hs = off_hx + (size_t)n * 8;
    const size_t off_st = off_hs + ((size_t)n * 4 + 255) / 256 * 256;
    const size_t off_hist = off_st + 2 * sizeof(SelectState);
    const size_t off_lam = off_hist + 512 * 4;
    const size_t bytes = off_lam + 8;
    void* ws = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess) return BFGS_ERR_ALLOC;
    char* base = (char*)ws;
    double* wd = (double*)base;
    double* hx = (double*)(base + off_hx);
    float* hs = hs_out ? hs_out : (float*)(base + off_hs);
    SelectState* sel = (SelectState*)(base + off_st);
    uint32_t* hist = (uint32_t*)(base + off_hist);
    double* lam_d = (double*)(base + off_lam);
    int rc = BFGS_OK;
    if (hipMemcpyAsync(wd, w.data(), w.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) rc = BFGS_ERR_HIP;
    if (rc == BFGS_OK) {
        hipLaunchKernelGGL(smooth_x, dim3(grid_blocks(n)), dim3(256), 0, st, nx, nz * (int64_t)nparam, half, wd, hdiag,
                           hx);
        hipLaunchKernelGGL(smooth_z, dim3(grid_blocks(n)), dim3(256), 0, st, nx, nz, (int64_t)nparam, half, wd, hx, hs);
        hipLaunchKernelGGL(select_init, dim3(1), dim3(256), 0, st, sel, (uint32_t)((n - 1) / 2), (uint32_t)(n / 2),
                           hist);
        for (int shift = 24; shift >= 0; shift -= 8) {
            hipLaunchKernelGGL(select_hist, dim3(grid_blocks(n)), dim3(256), 0, st, n, hs, sel, shift, hist);
            hipLaunchKernelGGL(select_pick, dim3(1), dim3(256), 0, st, sel, shift, hist);
        }
        hipLaunchKernelGGL(precond_finish, dim3(grid_blocks(n)), dim3(256), 0, st, n, hs, sel, damping, h0_out,
                           lam_d);
        if (hipGetLastError() != hipSuccess) rc = BFGS_ERR_HIP;
    }
    double lam = 0.0;
    if (rc == BFGS_OK && hipMemcpyAsync(&lam, lam_d, 8, hipMemcpyDeviceToHost, st) != hipSuccess) rc = BFGS_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess && rc == BFGS_OK) rc = BFGS_ERR_HIP;
    (void)hipFree(ws);
    if (rc == BFGS_OK && lambda_out) *lambda_out = lam;
    return rc;
}
