// B_k V for a block of ncols vectors through the compact form of the inverse
// BFGS matrix (Byrd, Nocedal & Schnabel 1994), which reaches the eq. (3)
// recursion / Alg. 2 two-loop result with two streaming passes over S and Y
// instead of 2k sequential ones:
//
//   B_k = B_0 + [S  B_0 Y] [ R^-T (D + Y^T B_0 Y) R^-1   -R^-T ] [ S^T     ]
//                          [ -R^-1                        0    ] [ Y^T B_0 ]
//   with R = triu(S^T Y), D = diag(S^T Y).
//
// Pass 1 (gemm1):  Z = [S^T V ; Y^T (h0 o V)]          2k x c, float64 partials
// reduce:          fixed-order sum of the partials
// small solve:     P = R^-1 Z_s,  T = R^-T ((D + Y^T B_0 Y) P - Z_y)     (float64)
// Pass 2 (gemm2):  out = h0 o (V - Y P) + S T     (or - h0 o (Y P) + S T for B_k - B_0)
//
// This file holds the float64 matrix-core form of both passes (float32 and
// float64 storage, and bfloat16 where its own MFMA form in apply_mfma.hip does not
// apply) and the inner solve shared by all forms.
#include <cmath>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

__global__ void reduce_partials(int64_t count, int nchunks, const double* __restrict__ part,
                                double* __restrict__ Z) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) s += part[(int64_t)ch * count + e];
    Z[e] = s;
}

// One 64-lane wave per probe column j.
//   P = R^-1 Z_s               (column-oriented back substitution)
//   W = (D + YHY) P - Z_y
//   T = R^-T W                 (row-oriented forward substitution)
// Rm is column-major with leading dimension kmax: R(l, i) = Rm[i * kmax + l].
constexpr int SOLVE_MAXK_PER_LANE = BFGS_MAX_PAIRS / 64;

__global__ void __launch_bounds__(64) small_solve(int k, int kmax, int c, const double* __restrict__ Rm,
                                                  const double* __restrict__ YHY, const double* __restrict__ Z,
                                                  double* __restrict__ P, double* __restrict__ T,
                                                  int32_t* __restrict__ status) {
    extern __shared__ double sh[];
    double* b = sh;          // right-hand side, overwritten
    double* x = sh + k;      // P column
    double* w = sh + 2 * k;  // W, then T column
    const int j = blockIdx.x, lane = threadIdx.x;
    const double* zs = Z + (int64_t)j * 2 * k;
    const double* zy = zs + k;
    for (int i = lane; i < k; i += 64) b[i] = zs[i];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double xi = b[i] / Rm[(int64_t)i * kmax + i];
        __syncthreads();
        if (lane == 0) x[i] = xi;
        for (int l = lane; l < i; l += 64) b[l] -= Rm[(int64_t)i * kmax + l] * xi;
        __syncthreads();
    }
    double acc[SOLVE_MAXK_PER_LANE];
#pragma unroll
    for (int u = 0; u < SOLVE_MAXK_PER_LANE; ++u) acc[u] = 0.0;
    for (int m = 0; m < k; ++m) {
        const double xm = x[m];
        const double* col = YHY + (int64_t)m * kmax;
#pragma unroll
        for (int u = 0; u < SOLVE_MAXK_PER_LANE; ++u) {
            const int l = lane + 64 * u;
            if (l < k) acc[u] = fma(col[l], xm, acc[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < SOLVE_MAXK_PER_LANE; ++u) {
        const int l = lane + 64 * u;
        if (l < k) w[l] = acc[u] + Rm[(int64_t)l * kmax + l] * x[l] - zy[l];
    }
    __syncthreads();
    for (int i = 0; i < k; ++i) {
        const double* col = Rm + (int64_t)i * kmax;
        double s = 0.0;
        for (int l = lane; l < i; l += 64) s = fma(col[l], w[l], s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        const double ti = (w[i] - s) / col[i];
        __syncthreads();
        if (lane == 0) w[i] = ti;
        __syncthreads();
    }
    bool bad = false;
    for (int i = lane; i < k; i += 64) {
        const double pv = x[i], tv = w[i];
        P[(int64_t)j * k + i] = pv;
        T[(int64_t)j * k + i] = tv;
        bad |= !isfinite(pv) || !isfinite(tv);
    }
    if (bad) set_status(status, BFGS_ERR_NONFINITE);
}

// Same solve through the stored R^-1, for k <= 256: one workgroup per block of 8
// probe columns, one thread per pair index.
//   P = R^-1 Z_s;  W = (D + YHY) P - Z_y;  T = R^-T W
constexpr int SB_COLS = 4;

__device__ __forceinline__ void small_solve_block(int k, int kmax, int c, const double* __restrict__ Rm,
                                                  const double* __restrict__ Rinv, const double* __restrict__ RinvT,
                                                  const double* __restrict__ YHY, const double* __restrict__ Z,
                                                  double* __restrict__ P, double* __restrict__ T,
                                                  int32_t* __restrict__ status, int blk) {
    __shared__ double a_sh[256][SB_COLS + 1];
    __shared__ double b_sh[256][SB_COLS + 1];
    const int i = threadIdx.x;
    const int j0 = blk * SB_COLS;
    const int nj = min(SB_COLS, c - j0);
    for (int e = threadIdx.x; e < k * SB_COLS; e += blockDim.x) {
        const int l = e % k, jj = e / k;
        a_sh[l][jj] = jj < nj ? Z[(int64_t)(j0 + jj) * 2 * k + l] : 0.0;
        b_sh[l][jj] = jj < nj ? Z[(int64_t)(j0 + jj) * 2 * k + k + l] : 0.0;
    }
    __syncthreads();
    double acc[SB_COLS];
#pragma unroll
    for (int jj = 0; jj < SB_COLS; ++jj) acc[jj] = 0.0;
    if (i < k)
#pragma unroll 8
        for (int l = i; l < k; ++l) {
            const double r = Rinv[(int64_t)l * kmax + i];
#pragma unroll
            for (int jj = 0; jj < SB_COLS; ++jj) acc[jj] = fma(r, a_sh[l][jj], acc[jj]);
        }
    __syncthreads();
    if (i < k)
#pragma unroll
        for (int jj = 0; jj < SB_COLS; ++jj) a_sh[i][jj] = acc[jj];   // P
    __syncthreads();
    if (i < k) {
        const double dii = Rm[(int64_t)i * kmax + i];
#pragma unroll
        for (int jj = 0; jj < SB_COLS; ++jj) acc[jj] = dii * a_sh[i][jj] - b_sh[i][jj];
#pragma unroll 8
        for (int l = 0; l < k; ++l) {
            const double y = YHY[(int64_t)l * kmax + i];
#pragma unroll
            for (int jj = 0; jj < SB_COLS; ++jj) acc[jj] = fma(y, a_sh[l][jj], acc[jj]);
        }
    }
    __syncthreads();
    if (i < k)
#pragma unroll
        for (int jj = 0; jj < SB_COLS; ++jj) b_sh[i][jj] = acc[jj];   // W
    __syncthreads();
    bool bad = false;
    if (i < k) {
#pragma unroll
        for (int jj = 0; jj < SB_COLS; ++jj) acc[jj] = 0.0;
#pragma unroll 8
        for (int l = 0; l <= i; ++l) {
            const double r = RinvT[(int64_t)l * kmax + i];
#pragma unroll
            for (int jj = 0; jj < SB_COLS; ++jj) acc[jj] = fma(r, b_sh[l][jj], acc[jj]);
        }
        for (int jj = 0; jj < nj; ++jj) {
            const double pv = a_sh[i][jj], tv = acc[jj];
            P[(int64_t)(j0 + jj) * k + i] = pv;
            T[(int64_t)(j0 + jj) * k + i] = tv;
            bad |= !isfinite(pv) || !isfinite(tv);
        }
    }
    if (bad) set_status(status, BFGS_ERR_NONFINITE);
    __syncthreads();   // a_sh and b_sh are free for the next block of columns
}

__global__ void __launch_bounds__(256) small_solve_blocks(int k, int kmax, int c, const double* __restrict__ Rm,
                                                          const double* __restrict__ Rinv,
                                                          const double* __restrict__ RinvT,
                                                          const double* __restrict__ YHY, const double* __restrict__ Z,
                                                          double* __restrict__ P, double* __restrict__ T,
                                                          int32_t* __restrict__ status) {
    small_solve_block(k, kmax, c, Rm, Rinv, RinvT, YHY, Z, P, T, status, blockIdx.x);
}

// k = 0: B_0 V (or zero for B_k - B_0); a non-finite input sets the deferred status.
template <typename Th, typename Tv, typename To>
__global__ void scale_by_h0(int64_t n, int c, const Th* __restrict__ h0, const Tv* __restrict__ V,
                            To* __restrict__ out, int diff, int32_t* __restrict__ status) {
    const int64_t total = n * c;
    bool bad = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % n;
        const double v = to_f64(h0[r]) * to_f64(V[e]);
        bad |= !isfinite(v);
        out[e] = diff ? (To)0 : (To)v;
    }
    if (bad) set_status(status, BFGS_ERR_NONFINITE);
}

// ---------------------------------------------------------------------------
// Float64 matrix-core forms of both passes for float32 and float64 storage
// (v_mfma_f64_16x16x4f64: lane l holds A(l % 16, l / 16), B(l / 16, l % 16) and
// C(l / 16 + 4 r, l % 16) in accumulator element r).  Both read W = [S | h0 o Y]
// (n x 2k), widened to float64 and scaled as it is staged:
//   pass 1:  Z = W^T V                  (= [S^T V ; Y^T (h0 o V)])
//   pass 2:  out = W [T ; -P] + h0 o V  (= h0 o (V - Y P) + S T; no h0 o V for B_k - B_0)
// Tiles are 128 x 128 on four waves (2 x 2, 4 x 4 fragments each); the next
// 16-deep stage is loaded into registers while the current one feeds the MFMAs.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int FT = 128;          // output tile edge
constexpr int FT_LD = FT + 4;    // LDS pitch of a staged row of 128
constexpr int FK = 16;           // reduction depth per stage

// Raw W entry (r, p) in the storage type: S's column p, or Y's column p - k (the h0
// factor of the Y half is applied when the value is staged).
template <typename Ts>
__device__ __forceinline__ Ts w_raw(const Ts* S, const Ts* Y, int64_t ld, int k, int p, int64_t r) {
    return p < k ? S[(int64_t)p * ld + r] : Y[(int64_t)(p - k) * ld + r];
}

// part[chunk][j * 2k + p] = sum over the chunk's rows of W(r, p) V(r, j); V's
// columns are ldv apart (n for a whole block; the block's row count when the rows
// come in slices).  Grid (nchunks, ceil(2k / 128), ceil(c / 128)).
template <typename Ts, typename Th, typename Tv>
__device__ __forceinline__ void gemm1_tile(int64_t n, int64_t ld, int k, int c, const Ts* __restrict__ S,
                                           const Ts* __restrict__ Y, const Th* __restrict__ h0,
                                           const Tv* __restrict__ V, int64_t ldv, double* __restrict__ part,
                                           int64_t rows_per_chunk, int bx, int by, int bz) {
    __shared__ double Ws[FK][FT_LD];
    __shared__ double Vs[FK][FT_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int twok = 2 * k;
    const int pi0 = by * FT, cj0 = bz * FT;
    const int64_t rb = (int64_t)bx * rows_per_chunk;
    const int64_t re = min(n, rb + rows_per_chunk);
    // staging map: element e = tid + 256 q (q < 8): row e % 16 (= tid % 16 for every q),
    // column e / 16; values stay in the storage type until they are staged
    Ts wreg[8];
    Tv vreg[8];
    double h0r = 0.0;
#define G1F_LOAD_STAGE(R0)                                                                   \
    {                                                                                      \
        const int64_t r = (R0) + tid % FK;                                                 \
        const bool rv = r < re;                                                            \
        h0r = rv ? to_f64(h0[r]) : 0.0;                                                    \
        _Pragma("unroll") for (int q = 0; q < 8; ++q) {                                    \
            const int cc = (tid + 256 * q) / FK;                                           \
            wreg[q] = (rv && pi0 + cc < twok) ? w_raw(S, Y, ld, k, pi0 + cc, r) : Ts{};     \
            vreg[q] = (rv && cj0 + cc < c) ? V[(int64_t)(cj0 + cc) * ldv + r] : Tv{};        \
        }                                                                                  \
    }
    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
    if (rb < re) { G1F_LOAD_STAGE(rb) }
    for (int64_t r0 = rb; r0 < re; r0 += FK) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q, rr = e % FK, cc = e / FK;
            const double w = to_f64(wreg[q]);
            Ws[rr][cc] = pi0 + cc < k ? w : w * h0r;
            Vs[rr][cc] = to_f64(vreg[q]);
        }
        __syncthreads();
        if (r0 + FK < re) { G1F_LOAD_STAGE(r0 + FK) }
#pragma unroll
        for (int kk = 0; kk < FK / 4; ++kk) {
            const int kr = 4 * kk + lane / 16, m = lane % 16;
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = Ws[kr][(wi * 4 + t) * 16 + m];
                b[t] = Vs[kr][(wj * 4 + t) * 16 + m];
            }
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = mfma64(a[ta], b[tb], acc[ta][tb]);
        }
        __syncthreads();
    }
#undef G1F_LOAD_STAGE
    double* dst = part + (int64_t)bx * twok * c;
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gp = pi0 + (wi * 4 + ta) * 16 + lane / 16 + 4 * r;
                const int gj = cj0 + (wj * 4 + tb) * 16 + lane % 16;
                if (gp < twok && gj < c) dst[(int64_t)gj * twok + gp] = acc[ta][tb][r];
            }
}

template <typename Ts, typename Th, typename Tv>
__global__ void __launch_bounds__(256, 2) gemm1_f64mfma(int64_t n, int64_t ld, int k, int c, const Ts* __restrict__ S,
                                                     const Ts* __restrict__ Y, const Th* __restrict__ h0,
                                                     const Tv* __restrict__ V, int64_t ldv, double* __restrict__ part,
                                                     int64_t rows_per_chunk) {
    gemm1_tile<Ts, Th, Tv>(n, ld, k, c, S, Y, h0, V, ldv, part, rows_per_chunk, blockIdx.x, blockIdx.y, blockIdx.z);
}

// out (column-major n x c, columns ldv apart, as V's) = W [T ; -P] (+ h0 o V unless
// diff); P, T column-major k x c.  Grid (ceil(n / 128), ceil(c / 128)).
template <typename Ts, typename Th, typename To, typename Tv>
__device__ __forceinline__ void gemm2_tile(int64_t n, int64_t ld, int k, int c, const Ts* __restrict__ S,
                                           const Ts* __restrict__ Y, const Th* __restrict__ h0,
                                           const Tv* __restrict__ V, int64_t ldv, const double* __restrict__ P,
                                           const double* __restrict__ T, To* __restrict__ out, int diff, int bx,
                                           int by) {
    __shared__ double stage_sh[FT * (FK + 1) + FK * FT_LD];
    double* Wsh = stage_sh;                     // [128 rows][FK + 1]
    double* Ms = stage_sh + FT * (FK + 1);      // [FK][FT_LD]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int twok = 2 * k;
    const int64_t row0 = (int64_t)bx * FT;
    const int col0 = by * FT;
    // W stage element e = tid + 256 q: row e % 128 (= tid % 128 for every q), pair
    // e / 128; M stage: pair e % 16, column e / 16
    Ts wreg[8];
    double mreg[8];
    const int64_t wr = row0 + tid % FT;
    const double h0w = wr < n ? to_f64(h0[wr]) : 0.0;
#define G2F_LOAD_STAGE(K0)                                                                       \
    _Pragma("unroll") for (int q = 0; q < 8; ++q) {                                            \
        const int e = tid + 256 * q;                                                           \
        const int kq = e / FT;                                                                 \
        wreg[q] = (wr < n && (K0) + kq < twok) ? w_raw(S, Y, ld, k, (K0) + kq, wr) : Ts{};      \
        const int pm = (K0) + e % FK, j = col0 + e / FK;                                       \
        double mv = 0.0;                                                                       \
        if (pm < twok && j < c) mv = pm < k ? T[(int64_t)j * k + pm] : -P[(int64_t)j * k + pm - k]; \
        mreg[q] = mv;                                                                          \
    }
    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
    G2F_LOAD_STAGE(0)
    for (int k0 = 0; k0 < twok; k0 += FK) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const double w = to_f64(wreg[q]);
            Wsh[(e % FT) * (FK + 1) + e / FT] = k0 + e / FT < k ? w : w * h0w;
            Ms[(e % FK) * FT_LD + e / FK] = mreg[q];
        }
        __syncthreads();
        if (k0 + FK < twok) { G2F_LOAD_STAGE(k0 + FK) }
#pragma unroll
        for (int kk = 0; kk < FK / 4; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = Wsh[((wi * 4 + t) * 16 + lane % 16) * (FK + 1) + 4 * kk + lane / 16];
                b[t] = Ms[(4 * kk + lane / 16) * FT_LD + (wj * 4 + t) * 16 + lane % 16];
            }
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = mfma64(a[ta], b[tb], acc[ta][tb]);
        }
        __syncthreads();
    }
#undef G2F_LOAD_STAGE
    // Transpose through LDS in groups of EC columns (Os[column][row], float64, so the
    // output is rounded once) so that each column's 128 rows are written, and V's
    // read, contiguously.
    constexpr int EC = 32;
    double* Os = stage_sh;
    static_assert(EC * (FT + 1) * sizeof(double) <= sizeof(stage_sh), "epilogue tile exceeds LDS");
    for (int g0 = 0; g0 < FT; g0 += EC) {
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) {
                const int jj = (wj * 4 + tb) * 16 + lane % 16 - g0;
                if (jj >= 0 && jj < EC) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rr = (wi * 4 + ta) * 16 + lane / 16 + 4 * r;
                        Os[jj * (FT + 1) + rr] = acc[ta][tb][r];
                    }
                }
            }
        __syncthreads();
        for (int e = tid; e < EC * FT; e += 256) {
            const int rr = e % FT, jj = e / FT;
            const int64_t r = row0 + rr;
            const int j = col0 + g0 + jj;
            if (r < n && j < c) {
                double o = Os[jj * (FT + 1) + rr];
                if (!diff) o += to_f64(h0[r]) * to_f64(V[(int64_t)j * ldv + r]);
                out[(int64_t)j * ldv + r] = (To)o;
            }
        }
        __syncthreads();
    }
}

template <typename Ts, typename Th, typename To, typename Tv>
__global__ void __launch_bounds__(256, 2) gemm2_f64mfma(int64_t n, int64_t ld, int k, int c, const Ts* __restrict__ S,
                                                     const Ts* __restrict__ Y, const Th* __restrict__ h0,
                                                     const Tv* __restrict__ V, int64_t ldv, const double* __restrict__ P,
                                                     const double* __restrict__ T, To* __restrict__ out, int diff) {
    gemm2_tile<Ts, Th, To, Tv>(n, ld, k, c, S, Y, h0, V, ldv, P, T, out, diff, blockIdx.x, blockIdx.y);
}

template <typename Ts, typename Th, typename To, typename Tv = Ts>
int apply_generic(bfgsuq_ctx* h, const void* Vv, int c, void* outv, bool diff, const ApplyWs* fixed) {
    const int64_t n = h->n;
    const int k = h->k;
    const Th* h0 = (const Th*)h->h0;
    const Tv* V = (const Tv*)Vv;
    To* out = (To*)outv;
    if (k == 0) {
        int64_t g = std::min<int64_t>(4096, (n * c + 255) / 256);
        hipLaunchKernelGGL((scale_by_h0<Th, Tv, To>), dim3((int)g), dim3(256), 0, h->stream, n, c, h0, V, out,
                           diff ? 1 : 0, h->status);
        return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
    }
    const int twok = 2 * k;
    const int ptiles = ceil_div(twok, FT), ctiles = ceil_div(c, FT);
    // row chunks: about 2048 pass-1 workgroups, each chunk a whole number of stages
    const int64_t max_chunks = std::max<int64_t>(1, (n + FK - 1) / FK);
    int nchunks = (int)std::min<int64_t>(max_chunks, std::max(1, 2048 / (ptiles * ctiles)));
    const size_t chunk_bytes = (size_t)twok * c * 8;
    if (fixed) {
        const int cap = (int)std::min<size_t>(fixed->part_bytes / chunk_bytes, 1 << 20);
        if (cap < 1) return BFGS_ERR_ARG;
        nchunks = std::min(nchunks, cap);
    }
    const int64_t rows_per_chunk = round_up((n + nchunks - 1) / nchunks, FK);
    nchunks = (int)((n + rows_per_chunk - 1) / rows_per_chunk);
    double *part, *Z, *P;
    if (fixed) {
        part = (double*)fixed->part;
        Z = fixed->Z;
        P = fixed->PT;
    } else {
        int rc;
        if ((rc = ensure_ws(h->part, (size_t)nchunks * chunk_bytes)) != BFGS_OK) return rc;
        if ((rc = ensure_ws(h->Z, (size_t)twok * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
        if ((rc = ensure_ws(h->PT, (size_t)2 * h->kmax * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
        part = (double*)h->part.ptr;
        Z = (double*)h->Z.ptr;
        P = (double*)h->PT.ptr;
    }
    double* T = P + (size_t)k * c;
    prof_begin(h, diff ? "hdiff_gemm1" : "apply_gemm1");
    hipLaunchKernelGGL((gemm1_f64mfma<Ts, Th, Tv>), dim3(nchunks, ptiles, ctiles), dim3(256), 0, h->stream, n, h->ld, k,
                       c, (const Ts*)h->S, (const Ts*)h->Y, h0, V, n, part, rows_per_chunk);
    const int64_t count = (int64_t)twok * c;
    prof_end(h);
    prof_begin(h, "apply_reduce");
    hipLaunchKernelGGL(reduce_partials, dim3(ceil_div(count, 256)), dim3(256), 0, h->stream, count, nchunks, part, Z);
    prof_end(h);
    if (int rc2 = apply_small_solve(h, c, Z, P, T)) return rc2;
    prof_begin(h, diff ? "hdiff_gemm2" : "apply_gemm2");
    hipLaunchKernelGGL((gemm2_f64mfma<Ts, Th, To, Tv>), dim3((unsigned)ceil_div(n, (int64_t)FT), ctiles), dim3(256), 0,
                       h->stream, n, h->ld, k, c, (const Ts*)h->S, (const Ts*)h->Y, h0, V, n, P, T, out,
                       diff ? 1 : 0);
    prof_end(h);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

// The same two passes for a history kept in host memory (bfgs_create_streamed): each
// pass streams S and Y through the device in row slices and runs its kernel on one
// slice while the next is copied; the pass-1 partials of all slices are summed in one
// fixed order, so the result does not depend on the copy timing.
template <typename Ts, typename Th, typename To, typename Tv = Ts>
int apply_streamed(bfgsuq_ctx* h, const void* Vv, int c, void* outv, bool diff) {
    const int64_t n = h->n;
    const int k = h->k;
    if (k == 0) return apply_generic<Ts, Th, To, Tv>(h, Vv, c, outv, diff, nullptr);   // reads no pair
    const Th* h0 = (const Th*)h->h0;
    const Tv* V = (const Tv*)Vv;
    To* out = (To*)outv;
    const int twok = 2 * k;
    const int ptiles = ceil_div(twok, FT), ctiles = ceil_div(c, FT);
    const int64_t sr = h->slice_rows;
    const int ns = (int)((n + sr - 1) / sr);
    int nsub = (int)std::min<int64_t>((sr + FK - 1) / FK, std::max(1, 2048 / (ptiles * ctiles)));
    const int64_t rows_per_sub = round_up((sr + nsub - 1) / nsub, FK);
    nsub = (int)((sr + rows_per_sub - 1) / rows_per_sub);
    const int64_t last_rows = n - (int64_t)(ns - 1) * sr;
    const int used = (ns - 1) * nsub + (int)((last_rows + rows_per_sub - 1) / rows_per_sub);
    const size_t chunk_bytes = (size_t)twok * c * 8;
    int rc;
    if ((rc = ensure_ws(h->part, (size_t)ns * nsub * chunk_bytes)) != BFGS_OK) return rc;
    if ((rc = ensure_ws(h->Z, (size_t)twok * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
    if ((rc = ensure_ws(h->PT, (size_t)2 * h->kmax * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
    double* part = (double*)h->part.ptr;
    double* Z = (double*)h->Z.ptr;
    double* P = (double*)h->PT.ptr;
    double* T = P + (size_t)k * c;
    {
        ProfScope ps(h, diff ? "hdiff_stream_pass1" : "apply_stream_pass1");
        rc = stream_slices(h, k, [&](int i, int64_t r0, int64_t rows, const void* Sst, const void* Yst) {
            const int nsi = (int)((rows + rows_per_sub - 1) / rows_per_sub);
            hipLaunchKernelGGL((gemm1_f64mfma<Ts, Th, Tv>), dim3(nsi, ptiles, ctiles), dim3(256), 0, h->stream, rows,
                               h->slice_ld, k, c, (const Ts*)Sst, (const Ts*)Yst, h0 + r0, V + r0, n,
                               part + (size_t)i * nsub * twok * c, rows_per_sub);
            return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
        });
        if (rc != BFGS_OK) return rc;
    }
    const int64_t count = (int64_t)twok * c;
    hipLaunchKernelGGL(reduce_partials, dim3(ceil_div(count, 256)), dim3(256), 0, h->stream, count, used, part, Z);
    if ((rc = apply_small_solve(h, c, Z, P, T)) != BFGS_OK) return rc;
    ProfScope ps(h, diff ? "hdiff_stream_pass2" : "apply_stream_pass2");
    rc = stream_slices(h, k, [&](int, int64_t r0, int64_t rows, const void* Sst, const void* Yst) {
        hipLaunchKernelGGL((gemm2_f64mfma<Ts, Th, To, Tv>), dim3((unsigned)ceil_div(rows, (int64_t)FT), ctiles),
                           dim3(256), 0, h->stream, rows, h->slice_ld, k, c, (const Ts*)Sst, (const Ts*)Yst, h0 + r0,
                           V + r0, n, P, T, out + r0, diff ? 1 : 0);
        return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
    });
    return rc;
}

// ---------------------------------------------------------------------------
// Persistent batched apply (float32 and float64 storage): the first pass of every
// problem, the float64 small steps of every problem and the second pass of every
// problem are one launch each.  A pass's workgroups take (problem, tile) items from
// a work queue (an atomic counter) until it runs dry; the problems are laid out
// longest first (work n k c), so the last items to be taken are small ones.  Each
// item is exactly one workgroup of the per-problem kernels (same tiles, same
// chunking, same fixed-order sums), so the results equal the per-problem path's.
// ---------------------------------------------------------------------------
template <typename Ts, typename Th, typename Tv>
__global__ void __launch_bounds__(256, 2) batch_pass1(const PersistProblem* __restrict__ pr, int nprob, int total,
                                                    unsigned* __restrict__ head) {
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item >= total) break;
        int lo = 0, hi = nprob - 1;   // last problem whose first item is <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pr[mid].first1 <= item) lo = mid;
            else hi = mid - 1;
        }
        const PersistProblem& q = pr[lo];
        const int local = item - q.first1, per = q.ptiles * q.ctiles;
        const int bx = local / per, rest = local % per;
        gemm1_tile<Ts, Th, Tv>(q.n, q.ld, q.k, q.c, (const Ts*)q.S, (const Ts*)q.Y, (const Th*)q.h0, (const Tv*)q.V,
                               q.n, q.part, q.rows_per_chunk, bx, rest % q.ptiles, rest / q.ptiles);
    }
}

// One workgroup per (problem, block of SB_COLS columns): the fixed-order sum of that
// block's pass-1 partials into Z, then the small solve of the block.
__global__ void __launch_bounds__(256) batch_solve(const PersistProblem* __restrict__ pr, int nprob) {
    int blk = blockIdx.x, p = 0;
    while (p < nprob && blk >= (pr[p].c + SB_COLS - 1) / SB_COLS) {
        blk -= (pr[p].c + SB_COLS - 1) / SB_COLS;
        ++p;
    }
    if (p >= nprob) return;   // whole workgroup
    const PersistProblem& q = pr[p];
    const int twok = 2 * q.k, j0 = blk * SB_COLS, nj = min(SB_COLS, q.c - j0);
    const int64_t count = (int64_t)twok * q.c;
    for (int e = threadIdx.x; e < twok * nj; e += blockDim.x) {
        const int64_t idx = (int64_t)j0 * twok + e;
        double sacc = 0.0;
        for (int ch = 0; ch < q.nchunks; ++ch) sacc += q.part[(int64_t)ch * count + idx];
        q.Z[idx] = sacc;
    }
    __threadfence_block();
    __syncthreads();
    small_solve_block(q.k, q.kmax, q.c, q.Rm, q.Rinv, q.RinvT, q.YHY, q.Z, q.P, q.P + (size_t)q.k * q.c, q.status,
                      blk);
}

template <typename Ts, typename Th, typename To, typename Tv>
__global__ void __launch_bounds__(256, 2) batch_pass2(const PersistProblem* __restrict__ pr, int nprob, int total,
                                                    unsigned* __restrict__ head) {
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item >= total) break;
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pr[mid].first2 <= item) lo = mid;
            else hi = mid - 1;
        }
        const PersistProblem& q = pr[lo];
        const int local = item - q.first2;
        gemm2_tile<Ts, Th, To, Tv>(q.n, q.ld, q.k, q.c, (const Ts*)q.S, (const Ts*)q.Y, (const Th*)q.h0,
                                   (const Tv*)q.V, q.n, q.P, q.P + (size_t)q.k * q.c, (To*)q.out, 0,
                                   local / q.ctiles, local % q.ctiles);
    }
}

// The work-queue heads start at zero for every launch (a kernel, so that a captured
// graph resets them on every replay).
__global__ void batch_reset(unsigned* __restrict__ head) {
    if (threadIdx.x < 2) head[threadIdx.x] = 0u;
}

template <typename Ts, typename Th>
int batch_persistent_impl(bfgsuq_ctx* const* hs, int nprob, const void* const* V, const int32_t* ncols,
                          void* const* out, hipStream_t st, PersistSlot* slot, bool upload, int wg_per_cu) {
    if (upload) {
        std::vector<int> order(nprob);
        for (int i = 0; i < nprob; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (double)hs[a]->n * hs[a]->k * ncols[a] > (double)hs[b]->n * hs[b]->k * ncols[b];
        });
        std::vector<PersistProblem> host(nprob);
        int t1 = 0, t2 = 0, tsolve = 0;
        for (int r = 0; r < nprob; ++r) {
            const int i = order[r];
            bfgsuq_ctx* h = hs[i];
            const int k = h->k, c = ncols[i], twok = 2 * k;
            if (k < 1 || k > 256) return BFGS_ERR_ARG;
            PersistProblem& q = host[r];
            q.n = h->n;
            q.ld = h->ld;
            q.k = k;
            q.kmax = h->kmax;
            q.c = c;
            q.S = h->S;
            q.Y = h->Y;
            q.h0 = h->h0;
            q.V = V[i];
            q.out = out[i];
            q.ptiles = ceil_div(twok, FT);
            q.ctiles = ceil_div(c, FT);
            // the per-problem path's chunking, so that the partial sums match it
            const int64_t max_chunks = std::max<int64_t>(1, (q.n + FK - 1) / FK);
            int nch = (int)std::min<int64_t>(max_chunks, std::max(1, 2048 / (q.ptiles * q.ctiles)));
            q.rows_per_chunk = round_up((q.n + nch - 1) / nch, FK);
            q.nchunks = (int)((q.n + q.rows_per_chunk - 1) / q.rows_per_chunk);
            int rc;
            if ((rc = ensure_ws(h->part, (size_t)q.nchunks * twok * c * 8)) != BFGS_OK) return rc;
            if ((rc = ensure_ws(h->Z, (size_t)twok * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
            if ((rc = ensure_ws(h->PT, (size_t)2 * h->kmax * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
            q.part = (double*)h->part.ptr;
            q.Z = (double*)h->Z.ptr;
            q.P = (double*)h->PT.ptr;
            q.Rm = h->Rm;
            q.Rinv = h->Rinv;
            q.RinvT = h->RinvT;
            q.YHY = h->YHY;
            q.status = h->status;
            q.first1 = t1;
            q.first2 = t2;
            t1 += q.nchunks * q.ptiles * q.ctiles;
            t2 += ceil_div(q.n, (int64_t)FT) * q.ctiles;
            tsolve += ceil_div(c, SB_COLS);
        }
        if (slot->cap < (size_t)nprob) {
            if (slot->prob) (void)hipFree(slot->prob);
            slot->prob = nullptr;
            slot->cap = 0;
            if (hipMalloc((void**)&slot->prob, (size_t)nprob * sizeof(PersistProblem)) != hipSuccess)
                return BFGS_ERR_ALLOC;
            slot->cap = (size_t)nprob;
        }
        if (!slot->head && hipMalloc((void**)&slot->head, 64) != hipSuccess) {
            slot->head = nullptr;
            return BFGS_ERR_ALLOC;
        }
        // pageable source: the call returns once the data is staged
        BFGS_HIP(hipMemcpyAsync(slot->prob, host.data(), (size_t)nprob * sizeof(PersistProblem),
                                hipMemcpyHostToDevice, st));
        slot->nprob = nprob;
        slot->items1 = t1;
        slot->items2 = t2;
        slot->solve_blocks = tsolve;
    }
    if (slot->nprob != nprob || !slot->prob) return BFGS_ERR_STATE;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int g1 = std::max(1, std::min(slot->items1, ncu * wg_per_cu));
    const int g2 = std::max(1, std::min(slot->items2, ncu * wg_per_cu));
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(64), 0, st, slot->head);
    hipLaunchKernelGGL((batch_pass1<Ts, Th, Ts>), dim3(g1), dim3(256), 0, st, slot->prob, nprob, slot->items1,
                       slot->head);
    hipLaunchKernelGGL(batch_solve, dim3(slot->solve_blocks), dim3(256), 0, st, slot->prob, nprob);
    hipLaunchKernelGGL((batch_pass2<Ts, Th, Th, Ts>), dim3(g2), dim3(256), 0, st, slot->prob, nprob, slot->items2,
                       slot->head + 1);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

}  // namespace

int batch_apply_persistent(bfgsuq_ctx* const* hs, int nprob, const void* const* V, const int32_t* ncols,
                           void* const* out, hipStream_t st, PersistSlot* slot, bool upload, int wg_per_cu) {
    if (nprob < 1) return BFGS_ERR_ARG;
    const bfgs_dtype s0 = hs[0]->storage;
    for (int i = 0; i < nprob; ++i)
        if (hs[i]->storage != s0 || hs[i]->streamed || hs[i]->k < 1 || hs[i]->k > 256) return BFGS_ERR_ARG;
    if (s0 == BFGS_F64) return batch_persistent_impl<double, double>(hs, nprob, V, ncols, out, st, slot, upload, wg_per_cu);
    if (s0 == BFGS_F32) return batch_persistent_impl<float, float>(hs, nprob, V, ncols, out, st, slot, upload, wg_per_cu);
    return BFGS_ERR_ARG;
}

int apply_small_solve(bfgsuq_ctx* h, int c, const double* Z, double* P, double* T) {
    ProfScope ps(h, "apply_solve");
    const int k = h->k;
    if (k <= 256)
        hipLaunchKernelGGL(small_solve_blocks, dim3(ceil_div(c, SB_COLS)), dim3(256), 0, h->stream, k, h->kmax, c,
                           h->Rm, h->Rinv, h->RinvT, h->YHY, Z, P, T, h->status);
    else
        hipLaunchKernelGGL(small_solve, dim3(c), dim3(64), 3 * k * sizeof(double), h->stream, k, h->kmax, c, h->Rm,
                           h->YHY, Z, P, T, h->status);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int apply_diff_float_block(bfgsuq_ctx* h, const void* V, bool v64, int32_t ncols, void* out, bool out64) {
    // (B_k - B_0) V for a float32 or float64 block V (a basis, not a probe block in the
    // storage type) on the float64 matrix cores, whatever the storage
    if (h->streamed) {
#define ADS(TS, TH)                                                                                      \
    if (v64 && out64) return apply_streamed<TS, TH, double, double>(h, V, ncols, out, true);           \
    if (v64) return apply_streamed<TS, TH, float, double>(h, V, ncols, out, true);                     \
    if (out64) return apply_streamed<TS, TH, double, float>(h, V, ncols, out, true);                   \
    return apply_streamed<TS, TH, float, float>(h, V, ncols, out, true);
        if (h->storage == BFGS_F64) { ADS(double, double) }
        if (h->storage == BFGS_F32) { ADS(float, float) }
#undef ADS
        return BFGS_ERR_ARG;
    }
#define ADF(TS, TH)                                                                                      \
    if (v64 && out64) return apply_generic<TS, TH, double, double>(h, V, ncols, out, true, nullptr);   \
    if (v64) return apply_generic<TS, TH, float, double>(h, V, ncols, out, true, nullptr);             \
    if (out64) return apply_generic<TS, TH, double, float>(h, V, ncols, out, true, nullptr);           \
    return apply_generic<TS, TH, float, float>(h, V, ncols, out, true, nullptr);
    switch (h->storage) {
        case BFGS_F64: { ADF(double, double) }
        case BFGS_F32: { ADF(float, float) }
        case BFGS_BF16: { ADF(bf16_t, float) }
    }
#undef ADF
    return BFGS_ERR_ARG;
}

int apply_block(bfgsuq_ctx* h, const void* V, int32_t ncols, void* out, bool diff, bool out64,
                const ApplyWs* fixed) {
    if (h->streamed) {
        // staged slices need the handle's own buffers: no fixed workspace
        if (fixed) return BFGS_ERR_STATE;
        if (h->storage == BFGS_F64 && !out64) return apply_streamed<double, double, double>(h, V, ncols, out, diff);
        if (h->storage == BFGS_F32)
            return out64 ? apply_streamed<float, float, double>(h, V, ncols, out, diff)
                         : apply_streamed<float, float, float>(h, V, ncols, out, diff);
        return BFGS_ERR_ARG;
    }
    if (out64) {
        if (h->storage != BFGS_F32) return BFGS_ERR_ARG;
        return apply_generic<float, float, double>(h, V, ncols, out, diff, fixed);
    }
    if (mfma_apply_supported(h, ncols)) return mfma_apply(h, V, ncols, out, diff, fixed);
    switch (h->storage) {
        case BFGS_F64: return apply_generic<double, double, double>(h, V, ncols, out, diff, fixed);
        case BFGS_F32: return apply_generic<float, float, float>(h, V, ncols, out, diff, fixed);
        case BFGS_BF16: return apply_generic<bf16_t, float, float>(h, V, ncols, out, diff, fixed);
    }
    return BFGS_ERR_ARG;
}
