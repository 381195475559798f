// Learned diagonal initial inverse Hessian: an 8 -> 64 -> 64 -> 1 GELU network
// predicting log h0 per (grid point, parameter) -- the learned counterpart of the
// paper's wavefield-based diagonal preconditioners (eqs. 4-8), with gamma I as
// the fallback when no network is used.
//
// Parameters (4801, flattened): W1 (64 x 8), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3.
// Float32 master copy, bfloat16 compute copy; every product accumulates in float32.
//
// Kernels: one wave per sample, lane = hidden unit.  The forward pass keeps the
// lane's rows of W1 and W2 in registers and exchanges activations through a
// per-wave LDS row; the backward pass accumulates the lane's gradient rows in
// registers and writes one partial gradient per wave, summed in a fixed order
// in float64 (deterministic), followed by Adam on the float32 master weights.
#include <cmath>
#include <new>

#include "common.h"

namespace {

constexpr int NP = 4801;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 4800;
constexpr int MLP_BLOCKS = 256;   // 4 waves each -> 1024 waves
constexpr int MLP_WAVES = MLP_BLOCKS * 4;

__device__ __forceinline__ float bfv(const uint16_t* w, int i) {
    bf16_t h;
    h.bits = w[i];
    return bf16_to_float(h);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// MODE 0: forward (out = network output), 1: forward + exp (h0), 2: loss gradient partials
template <int MODE>
__global__ void __launch_bounds__(256) mlp_kernel(const uint16_t* __restrict__ wbf, const float* __restrict__ X,
                                                  const float* __restrict__ target, int64_t N, float two_over_n,
                                                  float* __restrict__ out, float* __restrict__ partial) {
    __shared__ float W2s[64 * 64];
    __shared__ float hbuf[4][64];
    __shared__ float dbuf[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (MODE == 2)
        for (int e = threadIdx.x; e < 64 * 64; e += 256) W2s[e] = bfv(wbf, OFF_W2 + e);
    float w1[8], w2[64];
#pragma unroll
    for (int f = 0; f < 8; ++f) w1[f] = bfv(wbf, OFF_W1 + lane * 8 + f);
#pragma unroll
    for (int j = 0; j < 64; ++j) w2[j] = bfv(wbf, OFF_W2 + lane * 64 + j);
    const float b1 = bfv(wbf, OFF_B1 + lane), b2 = bfv(wbf, OFF_B2 + lane);
    const float w3 = bfv(wbf, OFF_W3 + lane), b3 = bfv(wbf, OFF_B3);
    float g1[8], g2[64];
#pragma unroll
    for (int f = 0; f < 8; ++f) g1[f] = 0.f;
#pragma unroll
    for (int j = 0; j < 64; ++j) g2[j] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
    __syncthreads();
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave, tw = (int64_t)gridDim.x * 4;
    for (int64_t s = gw; s < N; s += tw) {
        float x[8];
#pragma unroll
        for (int f = 0; f < 8; ++f) x[f] = X[s * 8 + f];
        float z1 = b1;
#pragma unroll
        for (int f = 0; f < 8; ++f) z1 = fmaf(w1[f], x[f], z1);
        const float h1 = gelu_f(z1);
        hbuf[wave][lane] = h1;
        __builtin_amdgcn_wave_barrier();
        float z2 = b2;
#pragma unroll
        for (int j = 0; j < 64; ++j) z2 = fmaf(w2[j], hbuf[wave][j], z2);
        const float h2 = gelu_f(z2);
        const float o = wave_sum(w3 * h2) + b3;
        if (MODE != 2) {
            if (lane == 0) out[s] = MODE == 1 ? expf(o) : o;
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        const float r = o - target[s];
        const float dout = r * two_over_n;
        if (lane == 0) {
            lsum = fmaf(r, r, lsum);
            gb3 += dout;
        }
        gw3 = fmaf(dout, h2, gw3);
        const float dz2 = dout * w3 * gelu_grad_f(z2);
        gb2 += dz2;
#pragma unroll
        for (int j = 0; j < 64; ++j) g2[j] = fmaf(dz2, hbuf[wave][j], g2[j]);
        dbuf[wave][lane] = dz2;
        __builtin_amdgcn_wave_barrier();
        float dh1 = 0.f;
#pragma unroll 16
        for (int l = 0; l < 64; ++l) dh1 = fmaf(W2s[l * 64 + lane], dbuf[wave][l], dh1);
        const float dz1 = dh1 * gelu_grad_f(z1);
        gb1 += dz1;
#pragma unroll
        for (int f = 0; f < 8; ++f) g1[f] = fmaf(dz1, x[f], g1[f]);
        __builtin_amdgcn_wave_barrier();
    }
    if (MODE != 2) return;
    float* P = partial + gw * (NP + 1);
#pragma unroll
    for (int f = 0; f < 8; ++f) P[OFF_W1 + lane * 8 + f] = g1[f];
    P[OFF_B1 + lane] = gb1;
#pragma unroll
    for (int j = 0; j < 64; ++j) P[OFF_W2 + lane * 64 + j] = g2[j];
    P[OFF_B2 + lane] = gb2;
    P[OFF_W3 + lane] = gw3;
    if (lane == 0) {
        P[OFF_B3] = gb3;
        P[NP] = lsum;
    }
}

// grad[p] = sum over waves (fixed order, float64); optional Adam step on the master weights.
__global__ void mlp_reduce_adam(const float* __restrict__ partial, int nwaves, float* __restrict__ grad,
                                float* __restrict__ loss, float* __restrict__ master, float* __restrict__ m1,
                                float* __restrict__ m2, uint16_t* __restrict__ wbf, int step, float lr, float inv_n,
                                int update) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    double g = 0.0;
    for (int w = 0; w < nwaves; ++w) g += (double)partial[(int64_t)w * (NP + 1) + p];
    if (p == NP) {
        if (loss) loss[0] = (float)(g * inv_n);
        return;
    }
    const float gf = (float)g;
    if (grad) grad[p] = gf;
    if (!update) return;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float a = beta1 * m1[p] + (1.f - beta1) * gf;
    const float b = beta2 * m2[p] + (1.f - beta2) * gf * gf;
    m1[p] = a;
    m2[p] = b;
    const float mhat = a / (1.f - powf(beta1, (float)step));
    const float vhat = b / (1.f - powf(beta2, (float)step));
    const float w = master[p] - lr * mhat / (sqrtf(vhat) + eps);
    master[p] = w;
    wbf[p] = float_to_bf16(w).bits;
}

__global__ void mlp_copy_params(const float* __restrict__ src, float* __restrict__ master, float* __restrict__ m1,
                                float* __restrict__ m2, uint16_t* __restrict__ wbf) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const float w = src[p];
    master[p] = w;
    m1[p] = 0.f;
    m2[p] = 0.f;
    wbf[p] = float_to_bf16(w).bits;
}

// Features of point i = (param p, iz, ix) of a field-major model vector.
__global__ void mlp_features_kernel(int64_t nx, int64_t nz, const float* __restrict__ logD,
                                    const float* __restrict__ gabs, float sigma_scale, float* __restrict__ X) {
    const int64_t m = nx * nz, n = 3 * m;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / m, r = i % m;
        const int64_t iz = r / nx;
        const int64_t q = (p + 1) % 3, u = (p + 2) % 3;
        float* f = X + i * 8;
        f[0] = logD[i];
        f[1] = logD[q * m + r];
        f[2] = logD[u * m + r];
        f[3] = gabs[i];
        f[4] = gabs[q * m + r];
        f[5] = gabs[u * m + r];
        f[6] = nz > 1 ? (float)iz / (float)(nz - 1) : 0.f;
        f[7] = sigma_scale;
    }
}

}  // namespace

struct bfgsuq_mlp {
    hipStream_t stream = nullptr;
    float* master = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    uint16_t* wbf = nullptr;
    float* partial = nullptr;
    int step = 0;
};

extern "C" {

int bfgs_mlp_destroy(bfgs_mlp_t m) {
    if (!m) return BFGS_OK;
    (void)hipStreamSynchronize(m->stream);
    void* ptrs[] = {m->master, m->m1, m->m2, m->wbf, m->partial};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
    return BFGS_OK;
}

int bfgs_mlp_create(void* stream, bfgs_mlp_t* out) {
    if (!out) return BFGS_ERR_ARG;
    *out = nullptr;
    bfgsuq_mlp* m = new (std::nothrow) bfgsuq_mlp();
    if (!m) return BFGS_ERR_ALLOC;
    m->stream = (hipStream_t)stream;
    if (hipMalloc(&m->master, NP * 4) != hipSuccess || hipMalloc(&m->m1, NP * 4) != hipSuccess ||
        hipMalloc(&m->m2, NP * 4) != hipSuccess || hipMalloc(&m->wbf, NP * 2) != hipSuccess ||
        hipMalloc(&m->partial, (size_t)MLP_WAVES * (NP + 1) * 4) != hipSuccess) {
        bfgs_mlp_destroy(m);
        return BFGS_ERR_ALLOC;
    }
    if (hipMemsetAsync(m->master, 0, NP * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->m1, 0, NP * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->m2, 0, NP * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->wbf, 0, NP * 2, m->stream) != hipSuccess || hipStreamSynchronize(m->stream) != hipSuccess) {
        bfgs_mlp_destroy(m);
        return BFGS_ERR_HIP;
    }
    *out = m;
    return BFGS_OK;
}

int bfgs_mlp_set_params(bfgs_mlp_t m, const float* params) {
    if (!m || !params) return BFGS_ERR_ARG;
    hipLaunchKernelGGL(mlp_copy_params, dim3((NP + 255) / 256), dim3(256), 0, m->stream, params, m->master, m->m1,
                       m->m2, m->wbf);
    m->step = 0;
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int bfgs_mlp_get_params(bfgs_mlp_t m, float* params) {
    if (!m || !params) return BFGS_ERR_ARG;
    BFGS_HIP(hipMemcpyAsync(params, m->master, NP * 4, hipMemcpyDeviceToDevice, m->stream));
    return BFGS_OK;
}

int bfgs_mlp_features(int64_t nx, int64_t nz, const float* logD, const float* gabs, float sigma_scale, float* X,
                      void* stream) {
    if (nx < 1 || nz < 1 || !logD || !gabs || !X) return BFGS_ERR_ARG;
    const int64_t n = 3 * nx * nz;
    const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(mlp_features_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, nx, nz, logD, gabs,
                       sigma_scale, X);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int bfgs_mlp_forward(bfgs_mlp_t m, const float* X, int64_t N, float* out, int32_t exp_out) {
    if (!m || !X || !out || N < 1) return BFGS_ERR_ARG;
    if (exp_out)
        hipLaunchKernelGGL(mlp_kernel<1>, dim3(MLP_BLOCKS), dim3(256), 0, m->stream, m->wbf, X, nullptr, N, 0.f, out,
                           nullptr);
    else
        hipLaunchKernelGGL(mlp_kernel<0>, dim3(MLP_BLOCKS), dim3(256), 0, m->stream, m->wbf, X, nullptr, N, 0.f, out,
                           nullptr);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

static int mlp_grad_impl(bfgs_mlp_t m, const float* X, const float* target, int64_t N, float* grad, float* loss,
                         float lr, int update) {
    hipLaunchKernelGGL(mlp_kernel<2>, dim3(MLP_BLOCKS), dim3(256), 0, m->stream, m->wbf, X, target, N,
                       (float)(2.0 / (double)N), nullptr, m->partial);
    if (update) ++m->step;
    hipLaunchKernelGGL(mlp_reduce_adam, dim3((NP + 1 + 255) / 256), dim3(256), 0, m->stream, m->partial, MLP_WAVES,
                       grad, loss, m->master, m->m1, m->m2, m->wbf, m->step, lr, (float)(1.0 / (double)N), update);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int bfgs_mlp_grad(bfgs_mlp_t m, const float* X, const float* target, int64_t N, float* grad, float* loss) {
    if (!m || !X || !target || N < 1) return BFGS_ERR_ARG;
    return mlp_grad_impl(m, X, target, N, grad, loss, 0.f, 0);
}

int bfgs_mlp_train_step(bfgs_mlp_t m, const float* X, const float* target, int64_t N, float lr, float* loss) {
    if (!m || !X || !target || N < 1 || !(lr > 0.f)) return BFGS_ERR_ARG;
    return mlp_grad_impl(m, X, target, N, nullptr, loss, lr, 1);
}

}  // extern "C"
