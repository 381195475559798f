// Single-pass randomized SVD of B_k - B_0 (Alg. 3) and the posterior variance
// of eqs. (10) and (14).
//
//   X = probes (c = rank + oversample columns)
//   E = (B_k - B_0) X                                  apply.hip, "difference" form
//   E = Q R                                            Householder TSQR (tsqr.hip)
//   Omega (Q^T X) = Q^T E = R                          LU with partial pivoting, float64
//   Omega <- (Omega + Omega^T) / 2;  Omega = U_s Lambda U_s^T     tridiagonal divide and conquer, float64
//   U = Q U_s[:, :rank],  Sigma = lambda[:rank],  d = h0 + sum_i lambda_i U_i^2
//
// Q^T E equals R exactly for E = Q R, so the R of the factorisation is used
// instead of a second product with E.  Q^T X and Q U_s run on the float64 matrix
// cores, except for bfloat16 storage, where they run on the bfloat16 matrix cores
// with Q and U_s split into bfloat16 terms (rsvd_bf16.hip).
#include <cmath>
#include <type_traits>
#include <utility>

#include "common.h"

int probes_launch(bfgsuq_ctx* h, uint64_t seed, int32_t c, void* X, hipStream_t stream);

namespace {

// 1 / sqrt(t) for t > 0, denormal t included (hardware estimate refined by two
// Newton steps).
__device__ __forceinline__ double rsqrt_refined(double t) {
    double y = __builtin_amdgcn_rsq(t);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double ty = t * y;
        const double e = fma(-ty, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// F = R2 R1 for upper-triangular row-major c x c factors.
__global__ void tri_mul(int c, const double* __restrict__ R2, const double* __restrict__ R1, double* __restrict__ F) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c * c; e += gridDim.x * blockDim.x) {
        const int i = e / c, j = e % c;
        double s = 0.0;
        for (int l = i; l <= j; ++l) s = fma(R2[(int64_t)i * c + l], R1[(int64_t)l * c + j], s);
        F[e] = s;
    }
}

__global__ void set_identity(double* __restrict__ M, int c) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c * c; e += gridDim.x * blockDim.x)
        M[e] = (e / c == e % c) ? 1.0 : 0.0;
}

__global__ void sum_chunks(int64_t count, int nchunks, const double* __restrict__ part, double* __restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) s += part[(int64_t)ch * count + e];
    out[e] = s;
}

// ---------------------------------------------------------------------------
// Small float64 steps, one workgroup of 256 threads.  Matrices live in global
// memory (at most 256 x 256 doubles, cache resident).
// ---------------------------------------------------------------------------
constexpr int SMALL_THREADS = 256;

template <int NTHR = SMALL_THREADS>
__device__ double wg_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NTHR / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// Float64 matrix-core kernels (v_mfma_f64_16x16x4f64).  Fragment layout of one
// 16 x 16 x 4 product C += A B on a wave: lane l holds A(l % 16, l / 16),
// B(l / 16, l % 16), and C(l / 16 + 4 r, l % 16) in accumulator element r.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Both kernels below are 128 x 128 output tiles per workgroup, 2 x 2 waves of
// 4 x 4 fragments each, with the next operand stage loaded into registers while
// the current one (in LDS) feeds the matrix cores.
constexpr int MT_TILE = 128;
constexpr int MT_LD = MT_TILE + 4;
constexpr int MT_K = 16;          // reduction depth staged per step

// part[ch] = Q[rows of chunk ch, :]^T X[rows of chunk ch, :]  (cq x cx, column-major:
// part[j * cq + i] = sum_r Q(r, i) X(r, j)), Q column-major n x cq, X n x cx (both
// leading dimension n).  Grid (nchunk, ceil(cq / 128), ceil(cx / 128)): workgroup
// (ch, bi, bj) owns output rows bi * 128.. and columns bj * 128..
template <typename TQ, typename TX>
__global__ void __launch_bounds__(256, 2) qtx_mfma(int64_t n, int cq, int cx, const TQ* __restrict__ Q,
                                                const TX* __restrict__ X, double* __restrict__ part,
                                                int64_t rows_per_chunk) {
    __shared__ double Qs[MT_K][MT_LD];
    __shared__ double Xs[MT_K][MT_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int ci0 = blockIdx.y * MT_TILE, cj0 = blockIdx.z * MT_TILE;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_chunk;
    const int64_t re = min(n, rb + rows_per_chunk);
    // staging map: element e = tid + 256 q (q < 8): row e % 16, column e / 16
    TQ qreg[8];
    TX xreg[8];
#define QTX_LOAD_STAGE(R0)                                                                 \
    _Pragma("unroll") for (int q = 0; q < 8; ++q) {                                      \
        const int e = tid + 256 * q, rr = e % MT_K, cc = e / MT_K;                       \
        const int64_t r = (R0) + rr;                                                     \
        const bool rv = r < re;                                                          \
        qreg[q] = (rv && ci0 + cc < cq) ? Q[(int64_t)(ci0 + cc) * n + r] : TQ{};         \
        xreg[q] = (rv && cj0 + cc < cx) ? X[(int64_t)(cj0 + cc) * n + r] : TX{};         \
    }
    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
    if (rb < re) { QTX_LOAD_STAGE(rb) }
    for (int64_t r0 = rb; r0 < re; r0 += MT_K) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q, rr = e % MT_K, cc = e / MT_K;
            Qs[rr][cc] = to_f64(qreg[q]);
            Xs[rr][cc] = to_f64(xreg[q]);
        }
        __syncthreads();
        if (r0 + MT_K < re) { QTX_LOAD_STAGE(r0 + MT_K) }
#pragma unroll
        for (int kk = 0; kk < MT_K / 4; ++kk) {
            const int k = 4 * kk + lane / 16, m = lane % 16;
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = Qs[k][(wi * 4 + t) * 16 + m];
                b[t] = Xs[k][(wj * 4 + t) * 16 + m];
            }
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = mfma64(a[ta], b[tb], acc[ta][tb]);
        }
        __syncthreads();
    }
    double* out = part + (int64_t)blockIdx.x * cq * cx;
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = ci0 + (wi * 4 + ta) * 16 + lane / 16 + 4 * r;
                const int gj = cj0 + (wj * 4 + tb) * 16 + lane % 16;
                if (gi < cq && gj < cx) out[(int64_t)gj * cq + gi] = acc[ta][tb][r];
            }
}

// U = Q Us[:, :rank] (n x rank, column-major, TO) from column-major Q (n x c) and
// Us (column-major, leading dimension c); with SUB (float64 U) U -= Q Us instead.
// Grid (ceil(n / 128), ceil(rank / 128)).
template <typename TQ, typename TO, bool SUB = false>
__global__ void __launch_bounds__(256, 2) basis_mfma(int64_t n, int c, int rank, const TQ* __restrict__ Q,
                                                  const double* __restrict__ Us, TO* __restrict__ U) {
    __shared__ double stage_sh[MT_TILE * (MT_K + 1) + MT_K * MT_LD];
    double* Qs = stage_sh;                          // [128 rows][MT_K + 1]
    double* Ms = stage_sh + MT_TILE * (MT_K + 1);   // [MT_K][MT_LD]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    const int64_t row0 = (int64_t)blockIdx.x * MT_TILE;
    const int col0 = blockIdx.y * MT_TILE;
    TQ qreg[8];
    double mreg[8];
    // Q stage element e = tid + 256 q: row e % 128, k e / 128; Us stage: k e % 16, column e / 16
#define BASIS_LOAD_STAGE(K0)                                                                         \
    _Pragma("unroll") for (int q = 0; q < 8; ++q) {                                                \
        const int e = tid + 256 * q;                                                               \
        const int rr = e % MT_TILE, kq = e / MT_TILE;                                              \
        const int64_t r = row0 + rr;                                                               \
        qreg[q] = (r < n && (K0) + kq < c) ? Q[(int64_t)((K0) + kq) * n + r] : TQ{};               \
        const int km = e % MT_K, j = e / MT_K;                                                     \
        mreg[q] = ((K0) + km < c && col0 + j < rank) ? Us[(int64_t)(col0 + j) * c + (K0) + km] : 0.0; \
    }
    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
    BASIS_LOAD_STAGE(0)
    for (int k0 = 0; k0 < c; k0 += MT_K) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            Qs[(e % MT_TILE) * (MT_K + 1) + e / MT_TILE] = to_f64(qreg[q]);
            Ms[(e % MT_K) * MT_LD + e / MT_K] = mreg[q];
        }
        __syncthreads();
        if (k0 + MT_K < c) { BASIS_LOAD_STAGE(k0 + MT_K) }
#pragma unroll
        for (int kk = 0; kk < MT_K / 4; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = Qs[((wi * 4 + t) * 16 + lane % 16) * (MT_K + 1) + 4 * kk + lane / 16];
                b[t] = Ms[(4 * kk + lane / 16) * MT_LD + (wj * 4 + t) * 16 + lane % 16];
            }
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = mfma64(a[ta], b[tb], acc[ta][tb]);
        }
        __syncthreads();
    }
    if (sizeof(TO) == 4) {
        // transpose through LDS, one 64-column half at a time (64 x 129 floats fit in
        // the staging area): Os[column][row], then each column's 128 rows are contiguous
        float* Os = (float*)stage_sh;
        static_assert(64 * (MT_TILE + 1) * sizeof(float) <= sizeof(stage_sh), "epilogue tile exceeds LDS");
        for (int hh = 0; hh < 2; ++hh) {
            if (wj == hh) {
#pragma unroll
                for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                    for (int tb = 0; tb < 4; ++tb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = (wi * 4 + ta) * 16 + lane / 16 + 4 * r;
                            const int jj = tb * 16 + lane % 16;
                            Os[jj * (MT_TILE + 1) + rr] = (float)acc[ta][tb][r];
                        }
            }
            __syncthreads();
            for (int e = tid; e < 64 * MT_TILE; e += 256) {
                const int rr = e % MT_TILE, jj = e / MT_TILE;
                const int64_t r = row0 + rr;
                const int j = col0 + hh * 64 + jj;
                if (r < n && j < rank) U[(int64_t)j * n + r] = (TO)Os[jj * (MT_TILE + 1) + rr];
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + (wi * 4 + ta) * 16 + lane / 16 + 4 * r;
                    const int j = col0 + (wj * 4 + tb) * 16 + lane % 16;
                    if (j < rank && row < n) {
                        if (SUB) U[(int64_t)j * n + row] -= (TO)acc[ta][tb][r];
                        else U[(int64_t)j * n + row] = (TO)acc[ta][tb][r];
                    }
                }
    }
}

// Omega = F T^-1, symmetrised.  T column-major c x c (T[j*c + i] = T(i, j)).
// F = R, row-major c x c upper triangular.  Work: M = T^T (row-major M[i*c + j] =
// T(j, i) = T[i*c + j], i.e. the same array), B = F^T; solve M X = B, Omega = X^T.
//
// Blocked right-looking LU with partial pivoting in one workgroup: a panel of
// LU_NB columns is factored in LDS; each column of the rest of [M | B] then
// takes the panel's row swaps and the forward substitution with the panel's
// unit-lower block (one thread per column); the trailing rows are updated from
// the panel (L21) and the new U row block, both in LDS.  The backward
// substitution with U is blocked the same way.
// (value, index) of the largest value over a wave, ties to the lower index, in every
// lane (all lanes active).  Quad and 16-lane row steps by DPP, then the rows by the
// permlane swaps; each swap returns the lane's own pair and its partner's, and both
// are offered (the own one changes nothing).  The order does not matter: the
// selection is associative and commutative.
__device__ __forceinline__ void argmax_take(double& best, int& bi, double v, int i) {
    if (v > best || (v == best && i < bi)) {
        best = v;
        bi = i;
    }
}

template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double& best, int& bi) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, best);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    const int i2 = __builtin_amdgcn_update_dpp(0, bi, CTRL, 0xF, 0xF, false);
    argmax_take(best, bi, __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo), i2);
}

template <bool ROWS32>
__device__ __forceinline__ void argmax_swap(double& best, int& bi) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, best);
    const unsigned l0 = (unsigned)u, h0 = (unsigned)(u >> 32), i0 = (unsigned)bi;
    const auto lo = ROWS32 ? __builtin_amdgcn_permlane32_swap(l0, l0, false, false)
                           : __builtin_amdgcn_permlane16_swap(l0, l0, false, false);
    const auto hi = ROWS32 ? __builtin_amdgcn_permlane32_swap(h0, h0, false, false)
                           : __builtin_amdgcn_permlane16_swap(h0, h0, false, false);
    const auto ix = ROWS32 ? __builtin_amdgcn_permlane32_swap(i0, i0, false, false)
                           : __builtin_amdgcn_permlane16_swap(i0, i0, false, false);
#pragma unroll
    for (int t = 0; t < 2; ++t)
        argmax_take(best, bi, __builtin_bit_cast(double, ((unsigned long long)hi[t] << 32) | lo[t]), (int)ix[t]);
}

__device__ __forceinline__ void wave_argmax(double& best, int& bi) {
    argmax_dpp<0xB1>(best, bi);    // quad_perm [1, 0, 3, 2]
    argmax_dpp<0x4E>(best, bi);    // quad_perm [2, 3, 0, 1]
    argmax_dpp<0x124>(best, bi);   // row_ror:4
    argmax_dpp<0x128>(best, bi);   // row_ror:8
    argmax_swap<false>(best, bi);  // rows 0 <-> 1, 2 <-> 3
    argmax_swap<true>(best, bi);   // halves
}

constexpr int LU_NB = 16;
constexpr int LU_THREADS = 1024;
constexpr int LU_PLD = LU_NB + 1;        // panel row stride (doubles)
constexpr int LU_ULD = 2 * 256 + 1;      // row-block stride: M's right columns then B's columns

size_t omega_smem_bytes() { return ((size_t)256 * LU_PLD + (size_t)LU_NB * LU_ULD + LU_NB + 8) * sizeof(double); }

__global__ void __launch_bounds__(LU_THREADS) omega_solve(int c, double* __restrict__ M, const double* __restrict__ F,
                                                          double* __restrict__ B, double* __restrict__ Omega,
                                                          int* __restrict__ piv, int32_t* __restrict__ status) {
    extern __shared__ double lu_sh[];
    double* P = lu_sh;                              // panel rows kb..c-1: P[(r - kb) * LU_PLD + j]
    double* Ub = P + 256 * LU_PLD;                  // row block: Ub[i * LU_ULD + ec]
    double* red = Ub + LU_NB * LU_ULD;              // pivot value / index exchange
    __shared__ int pivl[LU_NB];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    // B(i, j) = F(j, i), row-major B[i*c + j]
    for (int e = tid; e < c * c; e += LU_THREADS) {
        const int i = e / c, j = e % c;
        B[e] = F[(int64_t)j * c + i];
    }
    __syncthreads();
    for (int kb = 0; kb < c; kb += LU_NB) {
        const int nb = min(LU_NB, c - kb);
        const int rows = c - kb;
        for (int e = tid; e < rows * nb; e += LU_THREADS) {
            const int r = e / nb, j = e % nb;
            P[r * LU_PLD + j] = M[(int64_t)(kb + r) * c + kb + j];
        }
        __syncthreads();
        // --- panel factorisation in LDS ---
        for (int j = 0; j < nb; ++j) {
            if (tid < 64) {
                double best = -1.0;
                int bi = j;
                for (int r = j + tid; r < rows; r += 64) {
                    const double v = fabs(P[r * LU_PLD + j]);
                    if (v > best) { best = v; bi = r; }
                }
                wave_argmax(best, bi);
                if (tid == 0) {
                    pivl[j] = bi;
                    piv[kb + j] = kb + bi;
                    if (!(best > 0.0) || !isfinite(best)) bad = 1;
                }
            }
            __syncthreads();
            const int p = pivl[j];
            if (p != j && tid < nb) {
                const double t = P[j * LU_PLD + tid];
                P[j * LU_PLD + tid] = P[p * LU_PLD + tid];
                P[p * LU_PLD + tid] = t;
            }
            __syncthreads();
            const double d = P[j * LU_PLD + j];
            for (int r = j + 1 + tid; r < rows; r += LU_THREADS) {
                const double l = d != 0.0 ? P[r * LU_PLD + j] / d : 0.0;
                P[r * LU_PLD + j] = l;
                for (int jj = j + 1; jj < nb; ++jj) P[r * LU_PLD + jj] = fma(-l, P[j * LU_PLD + jj], P[r * LU_PLD + jj]);
            }
            __syncthreads();
        }
        for (int e = tid; e < rows * nb; e += LU_THREADS) {
            const int r = e / nb, j = e % nb;
            M[(int64_t)(kb + r) * c + kb + j] = P[r * LU_PLD + j];
        }
        // --- swaps and forward substitution, one thread per column outside the panel ---
        // extended column ec: [0, kb) M left columns (swaps only); [kb + nb, c) M right
        // columns; then c columns of B
        const int right = c - kb - nb;
        for (int ec = tid; ec < kb + right + c; ec += LU_THREADS) {
            double* col;
            int stride = c;
            int ub = -1;
            if (ec < kb) {
                col = M + ec;
            } else if (ec < kb + right) {
                col = M + (kb + nb + (ec - kb));
                ub = ec - kb;
            } else {
                col = B + (ec - kb - right);
                ub = right + (ec - kb - right);
            }
            for (int j = 0; j < nb; ++j) {
                const int p = pivl[j];
                if (p != j) {
                    const double t = col[(int64_t)(kb + j) * stride];
                    col[(int64_t)(kb + j) * stride] = col[(int64_t)(kb + p) * stride];
                    col[(int64_t)(kb + p) * stride] = t;
                }
            }
            if (ub >= 0) {
                double x[LU_NB];
#pragma unroll
                for (int i = 0; i < LU_NB; ++i) {
                    if (i < nb) {
                        double v = col[(int64_t)(kb + i) * stride];
#pragma unroll
                        for (int l = 0; l < LU_NB; ++l)
                            if (l < i) v = fma(-P[i * LU_PLD + l], x[l], v);
                        x[i] = v;
                        col[(int64_t)(kb + i) * stride] = v;
                        Ub[i * LU_ULD + ub] = v;
                    }
                }
            }
        }
        __syncthreads();
        // --- trailing update of rows kb + nb .. c-1 over M's right columns and B:
        // C -= L21 U12, a rank-nb product on the float64 matrix cores, one wave per
        // 16 x 16 tile of C (A = L21 rows from the panel, B = U12 from the row block;
        // loads from clamped indices, stores only inside C) ---
        {
            const int trows = rows - nb;
            const int wcols = right + c;
            const int ntr = (trows + 15) / 16, ntc = (wcols + 15) / 16;
            const int lane = tid & 63, lm = lane & 15, lk = lane >> 4;
            for (int tile = tid >> 6; tile < ntr * ntc; tile += LU_THREADS / 64) {
                const int ti = tile / ntc, tj = tile % ntc;
                const int ec = tj * 16 + lm, ecc = min(ec, wcols - 1);
                double* colp = ecc < right ? M + (int64_t)(kb + nb) * c + kb + nb + ecc
                                           : B + (int64_t)(kb + nb) * c + (ecc - right);
                v4d acc;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = colp[(int64_t)min(ti * 16 + lk + 4 * q, trows - 1) * c];
                const int ar = min(ti * 16 + lm, trows - 1);
#pragma unroll
                for (int ks = 0; ks < LU_NB / 4; ++ks) {
                    const int k = 4 * ks + lk;
                    const double a = k < nb ? -P[(nb + ar) * LU_PLD + k] : 0.0;
                    const double b = k < nb ? Ub[k * LU_ULD + ecc] : 0.0;
                    acc = mfma64(a, b, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int rr = ti * 16 + lk + 4 * q;
                    if (rr < trows && ec < wcols) colp[(int64_t)rr * c] = acc[q];
                }
            }
        }
        __syncthreads();
    }
    // --- backward substitution U X = B, blocks from the bottom ---
    const int nblk = (c + LU_NB - 1) / LU_NB;
    for (int bidx = nblk - 1; bidx >= 0; --bidx) {
        const int kb = bidx * LU_NB;
        const int nb = min(LU_NB, c - kb);
        // U11 (nb x nb) into Ub's first rows; U[0:kb, kb:kb+nb] into P
        for (int e = tid; e < nb * nb; e += LU_THREADS) {
            const int i = e / nb, j = e % nb;
            Ub[i * LU_ULD + j] = M[(int64_t)(kb + i) * c + kb + j];
        }
        for (int e = tid; e < kb * nb; e += LU_THREADS) {
            const int r = e / nb, j = e % nb;
            P[r * LU_PLD + j] = M[(int64_t)r * c + kb + j];
        }
        __syncthreads();
        double* X = Ub + LU_NB;   // X[i * LU_ULD + col] for col < c (offset past U11's columns)
        for (int col = tid; col < c; col += LU_THREADS) {
            double x[LU_NB];
#pragma unroll
            for (int ii = LU_NB - 1; ii >= 0; --ii) {
                if (ii < nb) {
                    double v = B[(int64_t)(kb + ii) * c + col];
#pragma unroll
                    for (int l = 0; l < LU_NB; ++l)
                        if (l > ii && l < nb) v = fma(-Ub[ii * LU_ULD + l], x[l], v);
                    const double dii = Ub[ii * LU_ULD + ii];
                    v = dii != 0.0 ? v / dii : 0.0;
                    x[ii] = v;
                    B[(int64_t)(kb + ii) * c + col] = v;
                }
            }
#pragma unroll
            for (int ii = 0; ii < LU_NB; ++ii)
                if (ii < nb) X[ii * LU_ULD + col] = x[ii];
        }
        __syncthreads();
        // B[0:kb, :] -= U[0:kb, kb:kb+nb] X on the matrix cores, as above
        {
            const int ntr = (kb + 15) / 16, ntc = (c + 15) / 16;
            const int lane = tid & 63, lm = lane & 15, lk = lane >> 4;
            for (int tile = tid >> 6; tile < ntr * ntc; tile += LU_THREADS / 64) {
                const int ti = tile / ntc, tj = tile % ntc;
                const int col = tj * 16 + lm, colc = min(col, c - 1);
                v4d acc;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = B[(int64_t)min(ti * 16 + lk + 4 * q, kb - 1) * c + colc];
                const int ar = min(ti * 16 + lm, kb - 1);
#pragma unroll
                for (int ks = 0; ks < LU_NB / 4; ++ks) {
                    const int k = 4 * ks + lk;
                    const double a = k < nb ? -P[ar * LU_PLD + k] : 0.0;
                    const double b = k < nb ? X[k * LU_ULD + colc] : 0.0;
                    acc = mfma64(a, b, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = ti * 16 + lk + 4 * q;
                    if (r < kb && col < c) B[(int64_t)r * c + col] = acc[q];
                }
            }
        }
        __syncthreads();
    }
    // X = B (row-major); Omega = X^T; symmetrise.  Omega(i, j) = (X(j, i) + X(i, j)) / 2
    for (int e = tid; e < c * c; e += LU_THREADS) {
        const int i = e / c, j = e % c;
        const double v = 0.5 * (B[(int64_t)j * c + i] + B[(int64_t)i * c + j]);
        Omega[e] = v;
        if (!isfinite(v)) bad = 1;
    }
    __syncthreads();
    if (tid == 0 && bad) set_status(status, BFGS_ERR_NUMERIC);
}

// Symmetric eigendecomposition of A (row-major c x c, overwritten):
//   sym_tridiag        Householder tridiagonalisation (one workgroup); reflector kk
//                      (unit first entry, acting on rows kk+1..c-1) is stored
//                      contiguously at V[kk * c + r] with tau in taus[kk]
//   householder_accum  Z = H_0 H_1 ... H_{c-3} explicitly, one wave per column
//   tridiag_dc         eigenpairs of the tridiagonal (d, e) by divide and conquer,
//                      eigenvectors of A = Z times those of the tridiagonal
//                      (tridiag_dc.hip)
// Z: column-major c x c eigenvectors (Z[i*c + r] = component r of vector i).
// x summed over the wave, in every lane (all lanes active): quad and 16-lane row sums
// by DPP (quad permutations, row rotations by 4 and 8), then the four rows by the
// permlane swaps, which return across their two results each lane's own value and
// that of the same lane in the partner row.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double swap_sum16(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]) +
           __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}

__device__ __forceinline__ double swap_sum32(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]) +
           __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}

__device__ __forceinline__ double wave_sum_d(double x) {
    x += dpp_f64<0xB1>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_f64<0x124>(x);   // row_ror:4
    x += dpp_f64<0x128>(x);   // row_ror:8
    return swap_sum32(swap_sum16(x));
}

constexpr int TRI_THREADS = 1024;
constexpr int TRI_LDS_MAX = 191;   // trailing matrices up to this size run from LDS (packed lower triangle)
static_assert(TRI_LDS_MAX <= 193, "LDS-phase rows are covered by three 64-lane passes");

__host__ __device__ constexpr size_t tri_lds_bytes() { return (size_t)TRI_LDS_MAX * (TRI_LDS_MAX + 1) / 2 * 8; }

__device__ __forceinline__ int ptri(int i, int l) { return i * (i + 1) / 2 + l; }   // (i, l), l <= i

// Householder tridiagonalisation.  While the trailing matrix is larger than
// TRI_LDS_MAX the steps work on A in global memory (full symmetric storage); the
// remaining steps work on the packed lower triangle of A[b0:, b0:] in LDS, where
// the rank-2 update touches only the lower triangle.
__global__ void __launch_bounds__(TRI_THREADS) sym_tridiag(int c, double* __restrict__ A, double* __restrict__ V,
                                                             double* __restrict__ dg, double* __restrict__ eg,
                                                             double* __restrict__ taus) {
    extern __shared__ double Tl[];   // packed lower triangle of A[b0:, b0:]
    __shared__ double red[2 * (TRI_THREADS / 64)];
    __shared__ double vsh[256];
    __shared__ double wsh[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = TRI_THREADS / 64;
    const int b0 = c > TRI_LDS_MAX ? c - TRI_LDS_MAX : 0;
    for (int kk = 0; kk < b0 && kk + 2 < c; ++kk) {
        const int m = c - kk - 1;   // length of x = A(kk+1:, kk)
        double part = 0.0;
        for (int i = 1 + tid; i < m; i += TRI_THREADS) {
            const double x = A[(int64_t)(kk + 1 + i) * c + kk];
            part = fma(x, x, part);
        }
        const double xn2 = wg_sum<TRI_THREADS>(part, red);
        const double alpha = A[(int64_t)(kk + 1) * c + kk];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(fma(alpha, alpha, xn2)), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int i = tid; i < m; i += TRI_THREADS) {
            const double v = (i == 0) ? 1.0 : A[(int64_t)(kk + 1 + i) * c + kk] * scale;
            vsh[i] = v;
            V[(int64_t)kk * c + kk + 1 + i] = v;
        }
        __syncthreads();
        if (tid == 0) {
            taus[kk] = tau;
            dg[kk] = A[(int64_t)kk * c + kk];
            eg[kk] = beta;
        }
        if (tau != 0.0) {
            // p = tau * A22 v;  w = p - (tau/2)(p^T v) v;  A22 -= v w^T + w v^T
            // one wave per row, lanes across the row (coalesced), then a wave sum
            // two rows per pass, all loads of a pass first (m <= 255: four per lane and row)
            for (int i0 = wave; i0 < m; i0 += 2 * NW) {
                double sr[2] = {0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    const double* row = A + (int64_t)(kk + 1 + i) * c + (kk + 1);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int l = lane + 64 * u;
                        if (i < m && l < m) sr[r] = fma(row[l], vsh[l], sr[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    if (i >= m) break;   // uniform
                    const double p = wave_sum_d(sr[r]);
                    if (lane == 0) wsh[i] = tau * p;
                }
            }
            __syncthreads();
            double pp = 0.0;
            for (int i = tid; i < m; i += TRI_THREADS) pp = fma(wsh[i], vsh[i], pp);
            const double K = 0.5 * tau * wg_sum<TRI_THREADS>(pp, red);
            for (int i = tid; i < m; i += TRI_THREADS) wsh[i] -= K * vsh[i];
            __syncthreads();
            for (int i0 = wave; i0 < m; i0 += 2 * NW) {
                double x[2][4];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    const double* row = A + (int64_t)(kk + 1 + i) * c + (kk + 1);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int l = lane + 64 * u;
                        x[r][u] = (i < m && l < m) ? row[l] : 0.0;
                    }
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    if (i >= m) break;   // uniform
                    double* row = A + (int64_t)(kk + 1 + i) * c + (kk + 1);
                    const double vi = vsh[i], wi = wsh[i];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int l = lane + 64 * u;
                        if (l < m) row[l] = x[r][u] - (vi * wsh[l] + wi * vsh[l]);
                    }
                }
            }
        }
        __syncthreads();
    }
    // the trailing (c - b0) x (c - b0) matrix moves to LDS
    const int s0 = c - b0;
    for (int e = tid; e < s0 * (s0 + 1) / 2; e += TRI_THREADS) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (ptri(i + 1, 0) <= e) ++i;
        while (ptri(i, 0) > e) --i;
        const int l = e - ptri(i, 0);
        Tl[e] = A[(int64_t)(b0 + i) * c + b0 + l];
    }
    __syncthreads();
    // Three barriers per step: (v written) (p and the partials of p^T v written)
    // (A22 updated and the partials of the next column's norm written).  w = p - K v
    // is formed on the fly in the update, whose lane 0 of each row also sums the
    // squares of the next column below its subdiagonal.
    double* red2 = red + NW;
    double xn2 = 0.0;
    if (b0 + 2 < c) {
        const int m = c - b0 - 1;
        double part = 0.0;
        for (int i = 1 + tid; i < m; i += TRI_THREADS) {
            const double x = Tl[ptri(1 + i, 0)];
            part = fma(x, x, part);
        }
        xn2 = wg_sum<TRI_THREADS>(part, red);
    }
    for (int kk = b0; kk + 2 < c; ++kk) {
        const int o = kk - b0;      // local index of the column being eliminated
        const int m = c - kk - 1;
        const double alpha = Tl[ptri(o + 1, o)];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(fma(alpha, alpha, xn2)), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int i = tid; i < m; i += TRI_THREADS) {
            const double v = (i == 0) ? 1.0 : Tl[ptri(o + 1 + i, o)] * scale;
            vsh[i] = v;
            V[(int64_t)kk * c + kk + 1 + i] = v;
        }
        if (tid == 0) {
            taus[kk] = tau;
            dg[kk] = Tl[ptri(o, o)];
            eg[kk] = beta;
        }
        __syncthreads();
        const int q0 = o + 1;
        if (tau != 0.0) {
            // p_i = tau sum_l A22(i, l) v_l: row i up to the diagonal, then column i below
            // it; each wave also sums p_i v_i over its rows
            double pv = 0.0, vl[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int l = lane + 64 * u;
                vl[u] = l < m ? vsh[l] : 0.0;
            }
            for (int i0 = wave; i0 < m; i0 += 2 * NW) {
                double sr[2] = {0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW, gi = q0 + i, rbase = ptri(gi, q0);
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int l = lane + 64 * u;
                        const double aval = (i < m && l < m) ? (l <= i ? Tl[rbase + l] : Tl[ptri(q0 + l, gi)]) : 0.0;
                        sr[r] = fma(aval, vl[u], sr[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    if (i >= m) break;   // uniform
                    const double p = tau * wave_sum_d(sr[r]);
                    if (lane == 0) wsh[i] = p;
                    pv = fma(p, vsh[i], pv);
                }
            }
            if (lane == 0) red[wave] = pv;
            __syncthreads();
            double ps = 0.0;
            for (int w = 0; w < NW; ++w) ps += red[w];
            const double K = 0.5 * tau * ps;
            // lower triangle of A22 -= v w^T + w v^T with w = p - K v; two rows per pass,
            // every load of a pass issued before its stores (rows do not overlap, which
            // the compiler cannot see)
            double nrm = 0.0;
            for (int i0 = wave; i0 < m; i0 += 2 * NW) {
                double x[2][3], vl[3], wl[3];
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const int l = lane + 64 * u;
                    vl[u] = l < m ? vsh[l] : 0.0;
                    wl[u] = l < m ? fma(-K, vl[u], wsh[l]) : 0.0;
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    const double* row = Tl + ptri(q0 + i, q0);
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int l = lane + 64 * u;
                        x[r][u] = (i < m && l <= i) ? row[l] : 0.0;
                    }
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int i = i0 + r * NW;
                    if (i >= m) break;   // uniform
                    double* row = Tl + ptri(q0 + i, q0);
                    const double vi = vsh[i], wi = fma(-K, vi, wsh[i]);
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int l = lane + 64 * u;
                        if (l <= i) {
                            const double y = x[r][u] - (vi * wl[u] + wi * vl[u]);
                            row[l] = y;
                            if (l == 0 && i >= 2) nrm = fma(y, y, nrm);
                        }
                    }
                }
            }
            if (lane == 0) red2[wave] = nrm;
        } else {
            // A22 unchanged: the next column's norm directly
            double nrm = 0.0;
            for (int i = 2 + wave; i < m; i += NW)
                if (lane == 0) {
                    const double x = Tl[ptri(q0 + i, q0)];
                    nrm = fma(x, x, nrm);
                }
            if (lane == 0) red2[wave] = nrm;
        }
        __syncthreads();
        xn2 = 0.0;
        for (int w = 0; w < NW; ++w) xn2 += red2[w];
    }
    if (tid == 0) {
        if (c >= 2) {
            dg[c - 2] = Tl[ptri(c - 2 - b0, c - 2 - b0)];
            eg[c - 2] = Tl[ptri(c - 1 - b0, c - 2 - b0)];
            taus[c - 2] = 0.0;
        }
        dg[c - 1] = Tl[ptri(c - 1 - b0, c - 1 - b0)];
        eg[c - 1] = 0.0;
    }
}

// Column col of Z = H_0 H_1 ... H_{c-3} e_col: the reflectors are applied to e_col
// from the last to the first.  One wave per column; lane holds rows lane + 64 q.
__global__ void __launch_bounds__(256) householder_accum(int c, const double* __restrict__ V,
                                                         const double* __restrict__ taus, double* __restrict__ Z) {
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= c) return;   // uniform per wave
    double z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) z[q] = (lane + 64 * q == col) ? 1.0 : 0.0;
    for (int kk = c - 3; kk >= 0; --kk) {
        const double tau = taus[kk];
        if (tau == 0.0) continue;
        double v[4];
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = lane + 64 * q;
            v[q] = (r > kk && r < c) ? V[(int64_t)kk * c + r] : 0.0;
            s = fma(v[q], z[q], s);
        }
        s = tau * wave_sum_d(s);
#pragma unroll
        for (int q = 0; q < 4; ++q) z[q] = fma(-s, v[q], z[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = lane + 64 * q;
        if (r < c) Z[(int64_t)col * c + r] = z[q];
    }
}

// Order eigenpairs by |lambda| descending (ties: lambda descending, then index),
// make each eigenvector's largest-magnitude entry positive (lowest index on ties),
// write lam_out (c) and Us (column-major c x c, sorted).
__global__ void __launch_bounds__(SMALL_THREADS) order_sign(int c, const double* __restrict__ d, const double* __restrict__ Z,
                                                            double* __restrict__ lam_out, double* __restrict__ Us) {
    __shared__ int dest[256];
    const int tid = threadIdx.x;
    for (int i = tid; i < c; i += SMALL_THREADS) {
        const double ai = fabs(d[i]), li = d[i];
        int rank = 0;
        for (int j = 0; j < c; ++j) {
            if (j == i) continue;
            const double aj = fabs(d[j]), lj = d[j];
            const bool before = (aj > ai) || (aj == ai && lj > li) || (aj == ai && lj == li && j < i);
            rank += before ? 1 : 0;
        }
        dest[i] = rank;
    }
    __syncthreads();
    for (int i = tid; i < c; i += SMALL_THREADS) {
        const int o = dest[i];
        lam_out[o] = d[i];
        const double* zc = Z + (int64_t)i * c;
        int arg = 0;
        double best = -1.0;
        for (int r = 0; r < c; ++r) {
            const double v = fabs(zc[r]);
            if (v > best) { best = v; arg = r; }
        }
        const double sg = zc[arg] < 0.0 ? -1.0 : 1.0;
        for (int r = 0; r < c; ++r) Us[(int64_t)o * c + r] = sg * zc[r];
    }
}

template <typename TO, typename Th>
__global__ void posterior_diag_kernel(int64_t n, int rank, const TO* __restrict__ U, const double* __restrict__ lam,
                                      const Th* __restrict__ h0, TO* __restrict__ dout, int32_t* __restrict__ status,
                                      int whitened) {
    // whitened basis (B_k = B_0 + B_0^1/2 U Lambda U^T B_0^1/2): d = h0 + h0 sum_i lam_i U_i^2
    bool bad = false;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const double hr = to_f64(h0[r]);
        double s = 0.0;
        for (int i = 0; i < rank; ++i) {
            const double u = to_f64(U[(int64_t)i * n + r]);
            s = fma(lam[i], u * u, s);
        }
        const TO d = (TO)(whitened ? fma(hr, s, hr) : hr + s);
        bad |= !isfinite(to_f64(d));
        dout[r] = d;
    }
    if (bad) set_status(status, BFGS_ERR_NONFINITE);   // includes overflow of the stored type
}

template <typename TO, typename Th>
__global__ void zero_rsvd(int64_t n, int rank, TO* __restrict__ U, double* __restrict__ Sigma, const Th* __restrict__ h0,
                          TO* __restrict__ dout) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * rank; e += (int64_t)gridDim.x * blockDim.x)
        U[e] = (TO)0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        dout[r] = (TO)to_f64(h0[r]);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < rank; i += blockDim.x) Sigma[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Column-blocked QR of a float64 E (n x c) when c is too wide for a float64 slot:
// E = [E1 E2] with E1 the first c1 columns; E1 = Q1 R11 (TSQR, two passes); E2 is
// projected off Q1 twice (block Gram-Schmidt with reorthogonalisation), R12 the sum
// of the two projections; the remainder = Q2 R22 (TSQR, two passes).  Then
// E = [Q1 Q2] [R11 R12; 0 R22].  Every block has c1, c - c1 <= 128 columns, whose
// slots are float64.
// ---------------------------------------------------------------------------
__global__ void add_into(int64_t count, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < count) dst[e] += src[e];
}

// R12 (column-major c1 x c2) += P (column-major c1 x c2) R22 (row-major c2 x c2, upper).
__global__ void add_p_times_r(int c1, int c2, const double* __restrict__ P, const double* __restrict__ R22,
                              double* __restrict__ R12) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c1 * c2; e += gridDim.x * blockDim.x) {
        const int i = e % c1, j = e / c1;
        double s = 0.0;
        for (int l = 0; l <= j; ++l) s = fma(P[(int64_t)l * c1 + i], R22[(int64_t)l * c2 + j], s);
        R12[e] += s;
    }
}

// R (row-major c x c) = [R11 R12; 0 R22]: R11 row-major c1 x c1, R12 column-major c1 x c2,
// R22 row-major c2 x c2.
__global__ void assemble_r(int c, int c1, const double* __restrict__ R11, const double* __restrict__ R12,
                           const double* __restrict__ R22, double* __restrict__ R) {
    const int c2 = c - c1;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c * c; e += gridDim.x * blockDim.x) {
        const int i = e / c, j = e % c;
        double v = 0.0;
        if (i < c1 && j < c1) v = R11[(int64_t)i * c1 + j];
        else if (i < c1) v = R12[(int64_t)(j - c1) * c1 + i];
        else if (j >= c1) v = R22[(int64_t)(i - c1) * c2 + (j - c1)];
        R[e] = v;
    }
}

// Two TSQR passes over one column block: src (n x cb) -> tmp -> dst; R (row-major cb x cb)
// = R2 R1 into Rout.
int tsqr_twice(bfgsuq_ctx* h, int cb, const double* src, double* tmp, double* dst, double* R1keep, double* Rout) {
    double* R = nullptr;
    int rc;
    if ((rc = tsqr_run(h, cb, src, tmp, &R)) != BFGS_OK) return rc;
    if (hipMemcpyAsync(R1keep, R, (size_t)cb * cb * 8, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        return BFGS_ERR_HIP;
    if ((rc = tsqr_run(h, cb, tmp, dst, &R)) != BFGS_OK) return rc;
    hipLaunchKernelGGL(tri_mul, dim3(ceil_div((int64_t)cb * cb, 256)), dim3(256), 0, h->stream, cb, R, R1keep, Rout);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int qr_two_blocks(bfgsuq_ctx* h, int c, double* E, double* Q, int nchunks, int64_t rows_per_chunk, double* part,
                  double* Rb, double* Rout) {
    const int64_t n = h->n;
    const int c1 = (int)std::min<int64_t>(128, round_up((c + 1) / 2, 16));
    const int c2 = c - c1;
    if (c2 < 1 || c2 > 128) return BFGS_ERR_ARG;
    int rc;
    if ((rc = ensure_ws(h->W, (size_t)n * c1 * 8)) != BFGS_OK) return rc;
    double* W = (double*)h->W.ptr;
    const size_t cc = (size_t)c * c;
    double* R11 = Rb;
    double* R12 = Rb + cc;
    double* R22 = Rb + 2 * cc;
    double* Rk = Rb + 3 * cc;   // first-pass R of a block, then one projection
    double* E2 = E + (int64_t)c1 * n;
    double* Q2 = Q + (int64_t)c1 * n;
    if ((rc = tsqr_twice(h, c1, E, W, Q, Rk, R11)) != BFGS_OK) return rc;
    const int64_t cnt = (int64_t)c1 * c2;
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL((qtx_mfma<double, double>), dim3(nchunks, ceil_div(c1, MT_TILE), ceil_div(c2, MT_TILE)),
                           dim3(256), 0, h->stream, n, c1, c2, Q, E2, part, rows_per_chunk);
        double* dst = pass == 0 ? R12 : Rk;
        hipLaunchKernelGGL(sum_chunks, dim3(ceil_div(cnt, 256)), dim3(256), 0, h->stream, cnt, nchunks, part, dst);
        hipLaunchKernelGGL((basis_mfma<double, double, true>), dim3((unsigned)ceil_div(n, (int64_t)MT_TILE),
                           ceil_div(c2, MT_TILE)), dim3(256), 0, h->stream, n, c1, c2, Q, dst, E2);
        if (pass == 1) hipLaunchKernelGGL(add_into, dim3(ceil_div(cnt, 256)), dim3(256), 0, h->stream, cnt, Rk, R12);
    }
    if ((rc = tsqr_twice(h, c2, E2, W, Q2, Rk, R22)) != BFGS_OK) return rc;
    // Where E2 lies in span(Q1) its remainder is rounding noise, which is not orthogonal
    // to Q1, and neither are the columns of Q2 it yields: project Q2 off Q1 once more and
    // refactor it.  Q2 = Q1 P + Q2', Q2' = Q2'' R'', so E2 = Q1 (R12 + P R22) + Q2'' (R'' R22).
    double* P = Rk;
    double* Rn = Rb + 4 * cc;
    double* Rn1 = Rb + 5 * cc;
    hipLaunchKernelGGL((qtx_mfma<double, double>), dim3(nchunks, ceil_div(c1, MT_TILE), ceil_div(c2, MT_TILE)),
                       dim3(256), 0, h->stream, n, c1, c2, Q, Q2, part, rows_per_chunk);
    hipLaunchKernelGGL(sum_chunks, dim3(ceil_div(cnt, 256)), dim3(256), 0, h->stream, cnt, nchunks, part, P);
    hipLaunchKernelGGL((basis_mfma<double, double, true>), dim3((unsigned)ceil_div(n, (int64_t)MT_TILE),
                       ceil_div(c2, MT_TILE)), dim3(256), 0, h->stream, n, c1, c2, Q, P, Q2);
    hipLaunchKernelGGL(add_p_times_r, dim3(ceil_div(cnt, 256)), dim3(256), 0, h->stream, c1, c2, P, R22, R12);
    if ((rc = tsqr_twice(h, c2, Q2, W, Q2, Rn1, Rn)) != BFGS_OK) return rc;
    hipLaunchKernelGGL(tri_mul, dim3(ceil_div((int64_t)c2 * c2, 256)), dim3(256), 0, h->stream, c2, Rn, R22, Rn1);
    R22 = Rn1;
    hipLaunchKernelGGL(assemble_r, dim3(ceil_div((int64_t)cc, 256)), dim3(256), 0, h->stream, c, c1, R11, R12, R22,
                       Rout);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

// Row scaling by h0^(p/2), p = +1 or -1 (the whitening of the preconditioned variant):
// in place, or into a copy.
template <typename T, typename Th>
__global__ void scale_rows_kernel(int64_t n, int c, const Th* __restrict__ h0, int p, const T* __restrict__ in,
                                  T* __restrict__ out) {
    const int64_t total = n * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const double hr = to_f64(h0[e % n]);
        const double w = p > 0 ? sqrt(hr) : 1.0 / sqrt(hr);
        out[e] = (T)(w * to_f64(in[e]));
    }
}

template <typename T>
void scale_rows_copy(bfgsuq_ctx* h, int c, const T* in, T* out, int p) {
    const int g = (int)std::min<int64_t>(8192, (h->n * c + 255) / 256);
    if (h->storage == BFGS_F64)
        hipLaunchKernelGGL((scale_rows_kernel<T, double>), dim3(g), dim3(256), 0, h->stream, h->n, c,
                           (const double*)h->h0, p, in, out);
    else
        hipLaunchKernelGGL((scale_rows_kernel<T, float>), dim3(g), dim3(256), 0, h->stream, h->n, c,
                           (const float*)h->h0, p, in, out);
}

template <typename T>
void scale_rows_launch(bfgsuq_ctx* h, int c, T* x, int p) {
    scale_rows_copy<T>(h, c, x, x, p);
}

// Omega = (M + M^T) / 2, column-major c x c.
__global__ void symmetrise(int c, const double* __restrict__ M, double* __restrict__ Om) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c * c; e += gridDim.x * blockDim.x) {
        const int i = e % c, j = e / c;
        Om[e] = 0.5 * (M[(int64_t)j * c + i] + M[(int64_t)i * c + j]);
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
template <typename TS, typename TO, typename Th>
int rsvd_impl(bfgsuq_ctx* h, int rank, int oversample, uint64_t seed, TO* U, double* Sigma, uint32_t flags) {
    const bool precond = (flags & BFGS_RSVD_PRECOND) != 0;
    const bool two_pass = (flags & BFGS_RSVD_TWO_PASS) != 0;
    const int64_t n = h->n;
    const int c = rank + oversample;
    int rc;
    if ((rc = ensure_ws(h->diag, (size_t)n * sizeof(TO))) != BFGS_OK) return rc;
    TO* dout = (TO*)h->diag.ptr;
    if (h->k == 0) {
        hipLaunchKernelGGL((zero_rsvd<TO, Th>), dim3(1024), dim3(256), 0, h->stream, n, rank, U, Sigma,
                           (const Th*)h->h0, dout);
        if (hipGetLastError() != hipSuccess) return BFGS_ERR_HIP;
        h->have_rsvd = true;
        h->last_rank = rank;
        return BFGS_OK;
    }
    if ((rc = ensure_ws(h->X, (size_t)n * c * sizeof(TS))) != BFGS_OK) return rc;
    // E = (B_k - B_0) X: float64 for float32 storage, whose Sigma would otherwise carry the
    // float32 rounding of E amplified by the Omega solve (about 6e-7 relative to Sigma_0
    // on the 1700 x 350 x 3 grid with k = 200, c = 220, against a 1e-6 budget)
    // and so is Q: rounding Q to float32 perturbs E = Q R by the same relative amount,
    // and with Q^T X built from the rounded Q the Omega solve amplifies it by cond(Q^T X)
    constexpr bool e64 = std::is_same<TS, float>::value;
    using TE = typename std::conditional<e64, double, TO>::type;
    using TQ = TE;
    if ((rc = ensure_ws(h->E, (size_t)n * c * sizeof(TE))) != BFGS_OK) return rc;
    // bfloat16 storage: Q chain-blocked (each TSQR chain's rows one contiguous block),
    // which the projection and the basis read without a translation miss per column;
    // the whitened and two-pass forms pass Q to column-major kernels and keep it so
    constexpr bool bf16_path = std::is_same<TS, bf16_t>::value;
    const bool qblk = bf16_path && !precond && !two_pass;
    const int64_t qb_rows = qblk ? tsqr_chain_rows(h) : 0;
    const int64_t q_rows = qblk ? ceil_div(n, qb_rows) * qb_rows : n;
    if ((rc = ensure_ws(h->Q, (size_t)q_rows * c * sizeof(TQ))) != BFGS_OK) return rc;
    // small: part(nchunks*c*c) + T, M, B, Omega, Z (5 c*c) + d, e, taus, rot, lam (5 c) + piv
    // Q^T X row chunks: about one per CU, each chunk a multiple of the staging depth
    int nchunks = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 63) / 64));
    const int64_t rows_per_chunk = round_up((n + nchunks - 1) / nchunks, MT_K);
    nchunks = (int)((n + rows_per_chunk - 1) / rows_per_chunk);
    // a blocked Q is projected one chain block per chunk
    const int qx_chunks = qblk ? (int)ceil_div(n, qb_rows) : nchunks;
    const int part_chunks = std::max(nchunks, qx_chunks);
    const size_t cc = (size_t)c * c;
    if ((rc = ensure_ws(h->small, ((size_t)part_chunks * cc + 14 * cc + 6 * (size_t)c) * 8 + (size_t)c * 4)) !=
        BFGS_OK)
        return rc;
    // tridiagonal eigensolver workspace, then Z = Q_H Y (c x c)
    const size_t ush_bytes = bf16_path ? basis_bf16_workspace(c, rank) : 0;
    const size_t ush_off = round_up((int64_t)(tridiag_dc_workspace(c) + cc * sizeof(double)), 256);
    if ((rc = ensure_ws(h->lam, ush_off + ush_bytes)) != BFGS_OK) return rc;
    double* dcwork = (double*)h->lam.ptr;
    double* Zt = dcwork + tridiag_dc_workspace(c) / sizeof(double);
    uint16_t* ush = (uint16_t*)((char*)h->lam.ptr + ush_off);   // 16-byte fragment loads
    double* part = (double*)h->small.ptr;
    double* Tm = part + (size_t)part_chunks * cc;
    double* Bm = Tm + cc;
    double* Om = Bm + cc;
    double* Zm = Om + cc;
    double* Usm = Zm + cc;
    double* dv = Usm + cc;
    double* ev = dv + c;
    double* tv = ev + c;
    double* rot = tv + c;
    double* lam = rot + 2 * (size_t)c;
    double* R1c = lam + c;
    double* Fm = R1c + cc;
    double* Rb = Fm + cc;   // 6 c x c: the column-blocked QR's pieces
    int* piv = (int*)(Rb + 6 * cc);
    TS* X = (TS*)h->X.ptr;
    TE* E = (TE*)h->E.ptr;
    TQ* Q = (TQ*)h->Q.ptr;

    {
        ProfScope ps(h, "probes");
        if ((rc = probes_launch(h, seed, c, X, h->stream)) != BFGS_OK) return rc;
    }
    if ((rc = apply_block(h, X, c, E, true, e64)) != BFGS_OK) return rc;
    // whitened operator B_0^-1/2 (B_k - B_0) B_0^-1/2: its sketch of X_w = B_0^1/2 X is
    // B_0^-1/2 E
    if (precond) scale_rows_launch(h, c, E, -1);
    double* R = nullptr;
    if constexpr (std::is_same<TE, double>::value) {
        if (tsqr_f64_slot(c)) {
            // E kept in float64 (float64 or float32 storage) is exactly rank deficient at
            // its noise level, and the zero-started slot then keeps part of Q.  A second
            // pass over the (well conditioned) Q restores orthonormality: E = Q2 (R2 R1).
            if ((rc = tsqr_run(h, c, E, Q, &R)) != BFGS_OK) return rc;
            if (hipMemcpyAsync(R1c, R, cc * 8, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) return BFGS_ERR_HIP;
            TQ* Q2 = reinterpret_cast<TQ*>(E);   // E is free now and as large as Q
            if ((rc = tsqr_run(h, c, Q, Q2, &R)) != BFGS_OK) return rc;
            hipLaunchKernelGGL(tri_mul, dim3(ceil_div((int64_t)cc, 256)), dim3(256), 0, h->stream, c, R, R1c, Fm);
            Q = Q2;
            R = Fm;
        } else {
            // wider than a float64 slot fits in LDS: two column blocks, each with a float64
            // slot (a float32 slot would round R at every fold)
            if ((rc = qr_two_blocks(h, c, E, Q, nchunks, rows_per_chunk, part, Rb, Fm)) != BFGS_OK) return rc;
            R = Fm;
        }
    } else {
        if constexpr (bf16_path) {
            if ((rc = tsqr_run(h, c, E, Q, &R, qblk)) != BFGS_OK) return rc;
        } else {
            if ((rc = tsqr_run(h, c, E, Q, &R)) != BFGS_OK) return rc;
        }
    }
    // the E / Q buffer that Q does not occupy is free now
    TE* Efree = (void*)Q == h->E.ptr ? (TE*)h->Q.ptr : E;
    if (two_pass) {
        // Halko et al.'s two-pass form: apply the operator to Q itself, Omega = Q^T (A Q)
        ProfScope ps(h, "two_pass_AQ");
        const TQ* V2 = Q;
        if (precond) {
            if ((rc = ensure_ws(h->W, (size_t)n * c * sizeof(TQ))) != BFGS_OK) return rc;
            TQ* Qs = (TQ*)h->W.ptr;
            scale_rows_copy(h, c, Q, Qs, -1);
            V2 = Qs;
        }
        if ((rc = apply_diff_float_block(h, V2, sizeof(TQ) == 8, c, Efree, sizeof(TE) == 8)) != BFGS_OK) return rc;
        if (precond) scale_rows_launch(h, c, Efree, -1);
        const int nblk = ceil_div(c, MT_TILE);
        hipLaunchKernelGGL((qtx_mfma<TQ, TE>), dim3(nchunks, nblk, nblk), dim3(256), 0, h->stream, n, c, c, Q, Efree,
                           part, rows_per_chunk);
        hipLaunchKernelGGL(sum_chunks, dim3(ceil_div((int64_t)cc, 256)), dim3(256), 0, h->stream, (int64_t)cc, nchunks,
                           part, Tm);
        hipLaunchKernelGGL(symmetrise, dim3(ceil_div((int64_t)cc, 256)), dim3(256), 0, h->stream, c, Tm, Om);
    } else {
        ProfScope ps(h, "proj_QtX");
        const TQ* Qp = Q;
        if (precond) {
            // T = Q^T X_w = (B_0^1/2 Q)^T X
            if ((rc = ensure_ws(h->W, (size_t)n * c * sizeof(TQ))) != BFGS_OK) return rc;
            TQ* Qs = (TQ*)h->W.ptr;
            scale_rows_copy(h, c, Q, Qs, +1);
            Qp = Qs;
        }
        if constexpr (bf16_path) {
            if ((rc = qtx_bf16_launch(h->stream, n, c, Qp, X, part, qx_chunks, qblk ? qb_rows : rows_per_chunk,
                                      qb_rows)) != BFGS_OK)
                return rc;
        } else {
            const int nblk = ceil_div(c, MT_TILE);
            hipLaunchKernelGGL((qtx_mfma<TQ, TS>), dim3(nchunks, nblk, nblk), dim3(256), 0, h->stream, n, c, c, Qp, X,
                               part, rows_per_chunk);
        }
        hipLaunchKernelGGL(sum_chunks, dim3(ceil_div((int64_t)cc, 256)), dim3(256), 0, h->stream, (int64_t)cc,
                           bf16_path ? qx_chunks : nchunks, part, Tm);
    }
    if (!two_pass) {
        ProfScope ps(h, "omega_lu");
        static bool attr = false;
        if (!attr) {
            if (hipFuncSetAttribute((const void*)omega_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)omega_smem_bytes()) != hipSuccess)
                return BFGS_ERR_HIP;
            attr = true;
        }
        hipLaunchKernelGGL(omega_solve, dim3(1), dim3(LU_THREADS), omega_smem_bytes(), h->stream, c, Tm, R, Bm, Om,
                           piv, h->status);
    }
    prof_begin(h, "sym_eig");
    // Bm (the LU right-hand sides) is free after omega_solve: it holds the reflectors
    {
        static bool attr = false;
        if (!attr) {
            if (hipFuncSetAttribute((const void*)sym_tridiag, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)tri_lds_bytes()) != hipSuccess)
                return BFGS_ERR_HIP;
            attr = true;
        }
        hipLaunchKernelGGL(sym_tridiag, dim3(1), dim3(TRI_THREADS), tri_lds_bytes(), h->stream, c, Om, Bm, dv, ev, tv);
    }
    hipLaunchKernelGGL(householder_accum, dim3(ceil_div(c, 4)), dim3(256), 0, h->stream, c, Bm, tv, Zm);
    double* wv = nullptr;
    if ((rc = tridiag_dc(h->stream, c, dv, ev, Zm, dcwork, &wv, Zt, h->status)) != BFGS_OK) return rc;
    hipLaunchKernelGGL(order_sign, dim3(1), dim3(SMALL_THREADS), 0, h->stream, c, wv, Zt, lam, Usm);
    if (hipMemcpyAsync(Sigma, lam, (size_t)rank * 8, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        return BFGS_ERR_HIP;
    prof_end(h);
    prof_begin(h, "basis_diag");
    if constexpr (bf16_path) {
        // the posterior diagonal is formed in the same pass
        if ((rc = basis_bf16_launch(h->stream, n, c, rank, Q, Usm, ush, lam, (const float*)h->h0, U, dout,
                                    h->status, precond, qb_rows)) != BFGS_OK)
            return rc;
    } else {
        hipLaunchKernelGGL((basis_mfma<TQ, TO>), dim3((unsigned)ceil_div(n, (int64_t)MT_TILE), ceil_div(rank, MT_TILE)),
                           dim3(256), 0, h->stream, n, c, rank, Q, Usm, U);
        const int g = (int)std::min<int64_t>(4096, (n + 255) / 256);
        hipLaunchKernelGGL((posterior_diag_kernel<TO, Th>), dim3(g), dim3(256), 0, h->stream, n, rank, U, lam,
                           (const Th*)h->h0, dout, h->status, precond ? 1 : 0);
    }
    prof_end(h);
    if (hipGetLastError() != hipSuccess) return BFGS_ERR_HIP;
    h->have_rsvd = true;
    h->last_rank = rank;
    return BFGS_OK;
}

}  // namespace

int rsvd_run(bfgsuq_ctx* h, int32_t rank, int32_t oversample, uint64_t seed, void* U, double* Sigma, uint32_t flags) {
    switch (h->storage) {
        case BFGS_F64: return rsvd_impl<double, double, double>(h, rank, oversample, seed, (double*)U, Sigma, flags);
        case BFGS_F32: return rsvd_impl<float, float, float>(h, rank, oversample, seed, (float*)U, Sigma, flags);
        case BFGS_BF16: return rsvd_impl<bf16_t, float, float>(h, rank, oversample, seed, (float*)U, Sigma, flags);
    }
    return BFGS_ERR_ARG;
}
