// The tall products of Alg. 3 for bfloat16 storage on the bfloat16 matrix cores
// (v_mfma_f32_32x32x16_bf16):
//   T = Q^T X           the projection (Q float32, X the bfloat16 probes)
//   U = Q Us[:, :rank]  the basis (Us the float64 eigenvectors), with the
//                       posterior diagonal of eqs. (10) and (14) in the same pass
//
// A value q is carried as three bfloat16 terms, q_hi = rne(q), q_mid =
// rne(q - q_hi), q_lo = rne(q - q_hi - q_mid), which hold a float32 value to
// 2^-25 (in practice exactly); bfloat16 products are exact in float32.
//   T = (Q_hi + Q_mid + Q_lo)^T X, X exact: each matrix-core step sums 16 exact
//       products in float32 and every 32 rows the float32 partial is added to
//       float64 accumulators, so T carries about one float32 rounding (Omega =
//       F T^-1 amplifies the rounding of T by about cond(T); float32 sums over
//       whole row chunks would grow with the chunk length).
//   U = Us_hi Q_hi + Us_hi Q_mid + Us_mid Q_hi + Us_hi Q_lo + Us_mid Q_mid + Us_lo Q_hi,
//       accumulated over c in float32 (the dropped products are below 2^-25).
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

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// q -> (hi, mid, lo) bfloat16 bit patterns
__device__ __forceinline__ void split_bits(float q, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
    const bf16_t h = float_to_bf16(q);
    const float r1 = q - bf16_to_float(h);
    const bf16_t m = float_to_bf16(r1);
    hi = h.bits;
    mid = m.bits;
    lo = float_to_bf16(r1 - bf16_to_float(m)).bits;
}

// eight float32 values -> hi, mid and lo fragments whose sum is exact: each term
// keeps the top 8 significant bits of what is left (truncation), and a float32
// significand has 24
__device__ __forceinline__ uint32_t top16(float x) { return __builtin_bit_cast(uint32_t, x) & 0xffff0000u; }

__device__ __forceinline__ void split8x3(const float (&q)[8], bf16x8& hi, bf16x8& mid, bf16x8& lo) {
    uint32_t h[4], m[4], l[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        uint32_t th[2], tm[2], tl[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float x = q[e + u];
            th[u] = top16(x);
            const float r1 = x - __builtin_bit_cast(float, th[u]);
            tm[u] = top16(r1);
            tl[u] = top16(r1 - __builtin_bit_cast(float, tm[u]));
        }
        h[e / 2] = (th[0] >> 16) | th[1];
        m[e / 2] = (tm[0] >> 16) | tm[1];
        l[e / 2] = (tl[0] >> 16) | tl[1];
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    mid = __builtin_bit_cast(bf16x8, make_uint4(m[0], m[1], m[2], m[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

// ---------------------------------------------------------------------------
// T = Q^T X.  Workgroup (chunk, jg) = one row chunk and the QX_NJ column tiles
// jg * QX_NJ .. of X; wave ti owns the 32-row block ti of T (columns 32 ti.. of Q).
// Q is column-major or chain-blocked (then a chunk is one block, its columns a few KB
// apart: the 32 columns a wave reads sit in one or two translation pages instead of
// 32, which cut the kernel from 2.3 to 1.6 ms at n = 1.785M, c = 220).
// The jgroups workgroups of a chunk sit on one XCD (workgroup g runs on XCD
// g % 8), so the chunk's Q rows come from HBM once.  Each 16-row step loads the
// lane's 8 rows of one Q column (32 bytes) and of QX_NJ X columns (16 bytes each)
// straight from HBM; steps alternate between two register sets.
// part[ch * c * c + j * c + i] = the chunk's float64 sums.
// ---------------------------------------------------------------------------
constexpr int QX_NJ = 2;
constexpr int QX_PF = 4;   // 16-row steps loaded ahead (even: the float64 flush is every second step)

struct QxStep {
    float q[8];
    uint4 x[QX_NJ];
    bool qv, xv[QX_NJ];   // row and column in range (out-of-range values are zeroed at use)
};

// Loads are unconditional, from addresses clamped into the arrays, so no branch
// separates a prefetch slot from its use and each step waits only for its own loads.
// qcol: the lane's column of Q (row r at qcol[r]).
template <bool VEC>
__device__ __forceinline__ void qx_load(QxStep& s, int64_t n, int c, const float* __restrict__ qcol,
                                        const bf16_t* __restrict__ X, int64_t row, int64_t rb, int64_t re, int icol,
                                        int jt0, int m) {
    // VEC: n % 8 == 0 and chunks end at multiples of 8, so a lane's 8 rows are all in
    // or all out, and re - 8 >= rb
    const int64_t rowc = min(row, re - 8 >= rb ? re - 8 : rb);
    s.qv = row < re && icol < c;
    if (VEC) {
        const float4* p = (const float4*)(qcol + rowc);
        const float4 a0 = p[0], a1 = p[1];
        s.q[0] = a0.x; s.q[1] = a0.y; s.q[2] = a0.z; s.q[3] = a0.w;
        s.q[4] = a1.x; s.q[5] = a1.y; s.q[6] = a1.z; s.q[7] = a1.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) s.q[e] = qcol[min(row + e, re - 1)];
    }
#pragma unroll
    for (int t = 0; t < QX_NJ; ++t) {
        const int jc = (jt0 + t) * 32 + m;
        s.xv[t] = row < re && jc < c;
        const int jcc = min(jc, c - 1);
        if (VEC) {
            s.x[t] = *(const uint4*)(X + (int64_t)jcc * n + rowc);
        } else {
            uint16_t b[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) b[e] = X[(int64_t)jcc * n + min(row + e, n - 1)].bits;
            s.x[t] = make_uint4(pack2(b[0], b[1]), pack2(b[2], b[3]), pack2(b[4], b[5]), pack2(b[6], b[7]));
        }
    }
}

// Rows past re are zeroed element by element in the scalar path (a lane's 8 rows can
// straddle re there).
template <bool VEC>
__device__ __forceinline__ void qx_mma(const QxStep& s, floatx16 (&acc)[QX_NJ], int64_t row, int64_t re) {
    float q[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) q[e] = (s.qv && (VEC || row + e < re)) ? s.q[e] : 0.f;
    bf16x8 hi, mid, lo;
    split8x3(q, hi, mid, lo);
#pragma unroll
    for (int t = 0; t < QX_NJ; ++t) {
        const uint4 xr = s.xv[t] ? s.x[t] : make_uint4(0, 0, 0, 0);
        const bf16x8 b = __builtin_bit_cast(bf16x8, xr);
        acc[t] = mma(lo, b, acc[t]);
        acc[t] = mma(mid, b, acc[t]);
        acc[t] = mma(hi, b, acc[t]);
    }
}

template <bool VEC>
__global__ void __launch_bounds__(512, 2) qtx_bf16(int64_t n, int c, const float* __restrict__ Q,
                                                   const bf16_t* __restrict__ X, double* __restrict__ part,
                                                   int nchunks, int64_t rows_per_chunk, int qblk) {
    const int lane = threadIdx.x & 63, half = lane >> 5, m = lane & 31;
    const int ntj = (c + 31) / 32, jgroups = (ntj + QX_NJ - 1) / QX_NJ;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const int chunk = (slot / jgroups) * 8 + xcd, jt0 = (slot % jgroups) * QX_NJ;
    if (chunk >= nchunks) return;   // whole workgroup (padding of the grid to 8 x jgroups)
    const int ti = threadIdx.x >> 6;
    const int icol = ti * 32 + m;
    const int64_t rb = (int64_t)chunk * rows_per_chunk;
    const int64_t re = min(n, rb + rows_per_chunk);
    // row r of column j at Qc[j * ldq + r]; out-of-range columns read the last one
    const float* Qc = qblk ? Q + (int64_t)chunk * rows_per_chunk * c - rb : Q;
    const int64_t ldq = qblk ? rows_per_chunk : n;
    const float* qcol = Qc + (int64_t)min(icol, c - 1) * ldq;
    floatx16 acc[QX_NJ];
    double accd[QX_NJ][16];
#pragma unroll
    for (int t = 0; t < QX_NJ; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            acc[t][i] = 0.f;
            accd[t][i] = 0.0;
        }
    // PF register slots of 16-row steps, each refilled after its step's products (the
    // compiler issues a pass's loads together; pinning each slot's loads right after its
    // products, so that more are in flight, measured slower).  The element-wise path
    // (n % 8 != 0) keeps two slots, which fit its registers.
    constexpr int PF = VEC ? QX_PF : 2;
    QxStep buf[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) qx_load<VEC>(buf[d], n, c, qcol, X, rb + 16 * d + 8 * half, rb, re, icol, jt0, m);
    for (int64_t r0 = rb; r0 < re; r0 += 16 * PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            qx_mma<VEC>(buf[d], acc, r0 + 16 * d + 8 * half, re);
            qx_load<VEC>(buf[d], n, c, qcol, X, r0 + 16 * (d + PF) + 8 * half, rb, re, icol, jt0, m);
            if (d & 1) {
                // the 32-row float32 partial into the float64 sums
#pragma unroll
                for (int t = 0; t < QX_NJ; ++t)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        accd[t][i] += (double)acc[t][i];
                        acc[t][i] = 0.f;
                    }
            }
        }
    }
    double* out = part + (int64_t)chunk * c * c;
#pragma unroll
    for (int t = 0; t < QX_NJ; ++t) {
        const int jc = (jt0 + t) * 32 + m;
        if (jt0 + t >= ntj || jc >= c) continue;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int ic = ti * 32 + 8 * (i / 4) + 4 * half + i % 4;
            if (ic < c) out[(int64_t)jc * c + ic] = accd[t][i];
        }
    }
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
                                                     float* __restrict__ dout, int32_t* __restrict__ status,
                                                     int whitened, int64_t qrb) {
    extern __shared__ uint16_t qs[];   // 2 * BS_BUF
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5;
    const bool mm = wave < (rank + 31) / 32;   // uniform per wave
    const int64_t r0 = (int64_t)blockIdx.x * BS_ROWS;
    // chain-blocked Q (qrb rows per block, qrb >= BS_ROWS / 2 and a multiple of 4): the
    // workgroup's rows lie in block b0 and at most the next one
    const int64_t b0 = qrb ? r0 / qrb : 0;
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
                const int64_t b = qrb ? b0 + (row - b0 * qrb >= qrb ? 1 : 0) : 0;
                const float* src = qrb ? Q + b * qrb * c + (int64_t)k * qrb + (row - b * qrb) : Q + (int64_t)k * n + row;
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
                // plain stores: streaming (non-temporal) ones made this pass 7 % slower and the
                // next apply 2 % slower
                if (j < rank && row < n) U[(int64_t)j * n + row] = acc[t][i];
            }
            sd += __shfl_xor(sd, 32, 64);   // the other half's columns of the same row
            if (half == 0) dpart[wave * BS_ROWS + t * 32 + lane] = sd;
        }
    }
    __syncthreads();
    const int nw = (rank + 31) / 32;
    bool bad = false;
    for (int rl = tid; rl < BS_ROWS; rl += nthr) {
        const int64_t row = r0 + rl;
        if (row >= n) continue;
        const double hr = (double)h0[row];
        double sd = 0.0;
        for (int w = 0; w < nw; ++w) sd += dpart[w * BS_ROWS + rl];
        // whitened basis: d = h0 + h0 sum_i lam_i U_i^2
        const float d = (float)(whitened ? fma(hr, sd, hr) : hr + sd);
        bad |= !isfinite(d);
        dout[row] = d;
    }
    if (bad) set_status(status, BFGS_ERR_NONFINITE);   // includes overflow of float32
}

}  // namespace

int qtx_bf16_launch(hipStream_t st, int64_t n, int c, const float* Q, const bf16_t* X, double* part, int nchunks,
                    int64_t rows_per_chunk, int64_t q_block) {
    if (c < 1 || c > 256 || rows_per_chunk % 16 != 0) return BFGS_ERR_ARG;
    // a blocked Q is read one block per chunk; every chunk holds at least one row
    if (q_block != 0 && (q_block != rows_per_chunk || (int64_t)(nchunks - 1) * rows_per_chunk >= n))
        return BFGS_ERR_ARG;
    const int qblk = q_block != 0 ? 1 : 0;
    const int ntj = (c + 31) / 32, jgroups = (ntj + QX_NJ - 1) / QX_NJ;
    const dim3 block(64 * ntj);   // <= 8 waves
    const dim3 grid((unsigned)(ceil_div((int64_t)nchunks, 8) * 8 * jgroups));
    if (n % 8 == 0)
        hipLaunchKernelGGL(qtx_bf16<true>, grid, block, 0, st, n, c, Q, X, part, nchunks, rows_per_chunk, qblk);
    else
        hipLaunchKernelGGL(qtx_bf16<false>, grid, block, 0, st, n, c, Q, X, part, nchunks, rows_per_chunk, qblk);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

size_t basis_bf16_workspace(int c, int rank) {
    const int nks = (c + 15) / 16, ntj = (rank + 31) / 32;
    return (size_t)ntj * nks * 3 * 512 * sizeof(uint16_t);
}

int basis_bf16_launch(hipStream_t st, int64_t n, int c, int rank, const float* Q, const double* Us, uint16_t* ush,
                      const double* lam, const float* h0, float* U, float* dout, int32_t* status, bool whitened,
                      int64_t q_block) {
    if (c < 1 || c > 256 || rank < 1 || rank > c) return BFGS_ERR_ARG;
    if (q_block != 0 && (q_block < BS_ROWS / 2 || q_block % 4 != 0)) return BFGS_ERR_ARG;
    const int nks = (c + 15) / 16, ntj = (rank + 31) / 32;
    const int total = ntj * nks * 512;
    hipLaunchKernelGGL(split_us, dim3((total + 255) / 256), dim3(256), 0, st, c, rank, nks, Us, ush);
    // enough waves that BS_PF float4 per thread stage BS_KC columns x BS_ROWS rows
    const int waves = std::max(ntj, BS_MIN_WAVES);
    static_assert(BS_PF * 64 * BS_MIN_WAVES >= BS_GROUPS, "staging map does not cover a stage");
    const dim3 grid((unsigned)((n + BS_ROWS - 1) / BS_ROWS)), block(64 * waves);
    const size_t smem = 2 * BS_BUF * sizeof(uint16_t);
    if (n % 4 == 0)
        hipLaunchKernelGGL(basis_bf16<true>, grid, block, smem, st, n, c, rank, nks, Q, ush, lam, h0, U, dout, status,
                           whitened ? 1 : 0, q_block);
    else
        hipLaunchKernelGGL(basis_bf16<false>, grid, block, smem, st, n, c, rank, nks, Q, ush, lam, h0, U, dout, status,
                           whitened ? 1 : 0, q_block);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}
