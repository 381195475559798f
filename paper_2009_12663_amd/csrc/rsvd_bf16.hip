// U = Q Us[:, :rank] of Alg. 3 for bfloat16 storage on the bfloat16 matrix cores
// (v_mfma_f32_32x32x16_bf16, float32 accumulation), with the posterior diagonal
// of eqs. (10) and (14) formed in the same pass.
//
// A value q is carried as three bfloat16 terms, q_hi = rne(q), q_mid =
// rne(q - q_hi), q_lo = rne(q - q_hi - q_mid), which hold a float32 value to
// 2^-25 (in practice exactly); bfloat16 products are exact in float32.
//   U = Us_hi Q_hi + Us_hi Q_mid + Us_mid Q_hi + Us_hi Q_lo + Us_mid Q_mid + Us_lo Q_hi,
//   accumulated over c in float32 (the dropped products are below 2^-25).
// The projection Q^T X is not done this way: Omega = F (Q^T X)^-1 amplifies the
// rounding of Q^T X by about its condition number, so its sums stay float64.
//
// Fragment layout of the 32x32x16 product C += A B on a wave: lane l holds
// A(l % 32, 8 (l / 32) + e) and B(8 (l / 32) + e, l % 32) for e = 0..7, and
// accumulator element i is C(8 (i / 4) + 4 (l / 32) + i % 4, l % 32).
#include <algorithm>

#include "common.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

__device__ __forceinline__ floatx16 mma(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// q -> (hi, mid, lo) bfloat16 bit patterns
__device__ __forceinline__ void split_bits(float q, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
    const bf16_t h = float_to_bf16(q);
    const float r1 = q - bf16_to_float(h);
    const bf16_t m = float_to_bf16(r1);
    hi = h.bits;
    mid = m.bits;
    lo = float_to_bf16(r1 - bf16_to_float(m)).bits;
}

// ---------------------------------------------------------------------------
// Us -> bfloat16 hi/mid/lo A fragments of U^T = Us^T Q^T: for column tile tj (32
// columns of Us) and 16-deep step ks, fragment p (0 hi, 1 mid, 2 lo) is 64 lanes
// x 8 values, lane (m, half) holding Us(16 ks + 8 half + e, 32 tj + m), zero
// outside c x rank.  Stored at ush[((tj * nks + ks) * 3 + p) * 512 + lane * 8 + e].
// ---------------------------------------------------------------------------
__global__ void split_us(int c, int rank, int nks, const double* __restrict__ Us, uint16_t* __restrict__ ush) {
    const int ntj = (rank + 31) / 32;
    const int total = ntj * nks * 64 * 8;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int e = idx % 8, lane = (idx / 8) % 64, f = idx / 512;
        const int ks = f % nks, tj = f / nks;
        const int k = 16 * ks + 8 * (lane >> 5) + e, j = 32 * tj + (lane & 31);
        // each term from the float64 residual of the ones before it
        const double dv = (k < c && j < rank) ? Us[(int64_t)j * c + k] : 0.0;
        const bf16_t h = float_to_bf16((float)dv);
        const double r1 = dv - (double)bf16_to_float(h);
        const bf16_t md = float_to_bf16((float)r1);
        const bf16_t l = float_to_bf16((float)(r1 - (double)bf16_to_float(md)));
        ush[((int64_t)f * 3 + 0) * 512 + lane * 8 + e] = h.bits;
        ush[((int64_t)f * 3 + 1) * 512 + lane * 8 + e] = md.bits;
        ush[((int64_t)f * 3 + 2) * 512 + lane * 8 + e] = l.bits;
    }
}

// ---------------------------------------------------------------------------
// U = Q Us[:, :rank], computed as U^T = Us^T Q^T so that a lane's accumulator
// column is one row of U (coalesced column-major writes).  Workgroup = BS_RT x 32
// rows of U, one wave per 32-column tile of U (at least BS_MIN_WAVES waves, the
// extra ones only stage).  The workgroup stages Q[rows, 32 columns] per stage (two 16-deep
// MFMA steps) through LDS as three bfloat16 planes ([row][32] each, double
// buffered); the next stage is loaded into registers while the current one feeds
// the matrix cores.  The A fragments come from split_us's array (L2 resident).
// ---------------------------------------------------------------------------
constexpr int BS_RT = 4;                    // 32-row tiles per workgroup
constexpr int BS_ROWS = 32 * BS_RT;
constexpr int BS_KC = 32;                   // Q columns per stage
constexpr int BS_LD = BS_KC + 8;            // LDS row pitch in bfloat16 (80 bytes)
constexpr int BS_PLANE = BS_ROWS * BS_LD;
constexpr int BS_BUF = 3 * BS_PLANE;        // hi, mid and lo planes of one stage (uint16)
constexpr int BS_GROUPS = BS_KC * BS_ROWS / 4;   // float4 groups per stage
constexpr int BS_PF = 3;                    // float4 groups per thread (>= BS_GROUPS / threads)
constexpr int BS_MIN_WAVES = 6;             // so that BS_PF * threads >= BS_GROUPS

template <bool VEC>
__global__ void __launch_bounds__(512, 4) basis_bf16(int64_t n, int c, int rank, int nks, const float* __restrict__ Q,
                                                     const uint16_t* __restrict__ ush, const double* __restrict__ lam,
                                                     const float* __restrict__ h0, float* __restrict__ U,
                                                     float* __restrict__ dout) {
    extern __shared__ uint16_t qs[];   // 2 * BS_BUF
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5;
    const bool mm = wave < (rank + 31) / 32;   // uniform per wave
    const int64_t r0 = (int64_t)blockIdx.x * BS_ROWS;
    const int nst = (c + BS_KC - 1) / BS_KC;
    // staging map: float4 group g = tid + q * nthr: column g % BS_KC, rows 4 (g / BS_KC) ..
    // (a wave's lanes cover 32 columns of two row groups: conflict-free LDS writes)
    float4 pre[BS_PF];
    auto load_stage = [&](int st) {
#pragma unroll
        for (int q = 0; q < BS_PF; ++q) {
            const int g = tid + q * nthr;
            const int k = st * BS_KC + g % BS_KC, rr = 4 * (g / BS_KC);
            const int64_t row = r0 + rr;
            float4 v = make_float4(0, 0, 0, 0);
            if (g < BS_GROUPS && k < c) {
                const float* src = Q + (int64_t)k * n + row;
                if (VEC) {
                    if (row < n) v = *(const float4*)src;   // n % 4 == 0: the group is all in or all out
                } else {
                    if (row < n) v.x = src[0];
                    if (row + 1 < n) v.y = src[1];
                    if (row + 2 < n) v.z = src[2];
                    if (row + 3 < n) v.w = src[3];
                }
            }
            pre[q] = v;
        }
    };
    auto store_stage = [&](int b) {
        uint16_t* hi = qs + b * BS_BUF;
#pragma unroll
        for (int q = 0; q < BS_PF; ++q) {
            const int g = tid + q * nthr;
            if (g >= BS_GROUPS) continue;
            const int k = g % BS_KC, rr = 4 * (g / BS_KC);
            const float v[4] = {pre[q].x, pre[q].y, pre[q].z, pre[q].w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                uint16_t h, md, l;
                split_bits(v[u], h, md, l);
                hi[(rr + u) * BS_LD + k] = h;
                hi[BS_PLANE + (rr + u) * BS_LD + k] = md;
                hi[2 * BS_PLANE + (rr + u) * BS_LD + k] = l;
            }
        }
    };
    floatx16 acc[BS_RT];
#pragma unroll
    for (int t = 0; t < BS_RT; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
    const uint4* afr = (const uint4*)ush + (int64_t)(mm ? wave : 0) * nks * 3 * 64 + lane;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int b = st & 1;
        if (st + 1 < nst) load_stage(st + 1);
        if (mm) {
            const uint16_t* hi = qs + b * BS_BUF;
#pragma unroll
            for (int kk = 0; kk < BS_KC / 16; ++kk) {
                const int ks = st * (BS_KC / 16) + kk;
                if (ks >= nks) break;   // uniform
                const bf16x8 ahi = __builtin_bit_cast(bf16x8, afr[(ks * 3 + 0) * 64]);
                const bf16x8 amd = __builtin_bit_cast(bf16x8, afr[(ks * 3 + 1) * 64]);
                const bf16x8 alo = __builtin_bit_cast(bf16x8, afr[(ks * 3 + 2) * 64]);
#pragma unroll
                for (int t = 0; t < BS_RT; ++t) {
                    const int off = (t * 32 + (lane & 31)) * BS_LD + kk * 16 + 8 * half;
                    const bf16x8 bhi = __builtin_bit_cast(bf16x8, *(const uint4*)(hi + off));
                    const bf16x8 bmd = __builtin_bit_cast(bf16x8, *(const uint4*)(hi + BS_PLANE + off));
                    const bf16x8 blo = __builtin_bit_cast(bf16x8, *(const uint4*)(hi + 2 * BS_PLANE + off));
                    // smallest terms first
                    acc[t] = mma(alo, bhi, acc[t]);
                    acc[t] = mma(amd, bmd, acc[t]);
                    acc[t] = mma(ahi, blo, acc[t]);
                    acc[t] = mma(amd, bhi, acc[t]);
                    acc[t] = mma(ahi, bmd, acc[t]);
                    acc[t] = mma(ahi, bhi, acc[t]);
                }
            }
        }
        if (st + 1 < nst) store_stage(b ^ 1);
        __syncthreads();
    }
    // U, and the posterior diagonal d = h0 + sum_j lambda_j U_j^2 (eqs. 10, 14) from
    // the stored float32 U: per wave over its columns in float64, then over the
    // waves in a fixed order (the staging LDS is free after the last barrier)
    double* dpart = (double*)qs;   // [wave][BS_ROWS]
    if (mm) {
        double lv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int j = wave * 32 + 8 * (i / 4) + 4 * half + i % 4;
            lv[i] = j < rank ? lam[j] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < BS_RT; ++t) {
            const int64_t row = r0 + t * 32 + (lane & 31);
            double sd = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int j = wave * 32 + 8 * (i / 4) + 4 * half + i % 4;
                const double u = (double)acc[t][i];
                sd = fma(lv[i], u * u, sd);
                // U is not read again here: streaming stores keep it out of the caches
                if (j < rank && row < n) __builtin_nontemporal_store(acc[t][i], U + (int64_t)j * n + row);
            }
            sd += __shfl_xor(sd, 32, 64);   // the other half's columns of the same row
            if (half == 0) dpart[wave * BS_ROWS + t * 32 + lane] = sd;
        }
    }
    __syncthreads();
    const int nw = (rank + 31) / 32;
    for (int rl = tid; rl < BS_ROWS; rl += nthr) {
        const int64_t row = r0 + rl;
        if (row >= n) continue;
        double sd = (double)h0[row];
        for (int w = 0; w < nw; ++w) sd += dpart[w * BS_ROWS + rl];
        dout[row] = (float)sd;
    }
}

}  // namespace

size_t basis_bf16_workspace(int c, int rank) {
    const int nks = (c + 15) / 16, ntj = (rank + 31) / 32;
    return (size_t)ntj * nks * 3 * 512 * sizeof(uint16_t);
}

int basis_bf16_launch(hipStream_t st, int64_t n, int c, int rank, const float* Q, const double* Us, uint16_t* ush,
                      const double* lam, const float* h0, float* U, float* dout) {
    if (c < 1 || c > 256 || rank < 1 || rank > c) return BFGS_ERR_ARG;
    const int nks = (c + 15) / 16, ntj = (rank + 31) / 32;
    const int total = ntj * nks * 512;
    hipLaunchKernelGGL(split_us, dim3((total + 255) / 256), dim3(256), 0, st, c, rank, nks, Us, ush);
    // enough waves that BS_PF float4 per thread stage BS_KC columns x BS_ROWS rows
    const int waves = std::max(ntj, BS_MIN_WAVES);
    static_assert(BS_PF * 64 * BS_MIN_WAVES >= BS_GROUPS, "staging map does not cover a stage");
    const dim3 grid((unsigned)((n + BS_ROWS - 1) / BS_ROWS)), block(64 * waves);
    const size_t smem = 2 * BS_BUF * sizeof(uint16_t);
    if (n % 4 == 0)
        hipLaunchKernelGGL(basis_bf16<true>, grid, block, smem, st, n, c, rank, nks, Q, ush, lam, h0, U, dout);
    else
        hipLaunchKernelGGL(basis_bf16<false>, grid, block, smem, st, n, c, rank, nks, Q, ush, lam, h0, U, dout);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}
