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
// This file holds the portable kernels that run every storage type with
// float64 accumulation; the bfloat16 form has MFMA kernels in apply_mfma.hip.
#include <cmath>

#include "common.h"

namespace {

constexpr int G1_TP = 64;   // pair-index tile
constexpr int G1_TC = 64;   // probe-column tile
constexpr int G1_TR = 32;   // rows per LDS stage

template <typename Ts, typename Th, typename Tv>
__global__ void __launch_bounds__(256) gemm1_generic(int64_t n, int64_t ld, int k, int c,
                                                     const Ts* __restrict__ S, const Ts* __restrict__ Y,
                                                     const Th* __restrict__ h0, const Tv* __restrict__ V,
                                                     double* __restrict__ part, int64_t rows_per_chunk) {
    __shared__ double As[G1_TR][G1_TP + 1];
    __shared__ double Bs[G1_TR][G1_TC + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int p0 = blockIdx.x * G1_TP, j0 = blockIdx.y * G1_TC;
    const int chunk = blockIdx.z;
    const int64_t r_begin = chunk * rows_per_chunk;
    const int64_t r_end = min(n, r_begin + rows_per_chunk);
    const int twok = 2 * k;
    double acc[4][4] = {};
    for (int64_t r0 = r_begin; r0 < r_end; r0 += G1_TR) {
        // A tile: pairs p0..p0+63 (S columns then h0-weighted Y columns), rows r0..r0+31
        for (int e = tid; e < G1_TR * G1_TP; e += 256) {
            const int rr = e % G1_TR, pp = e / G1_TR;
            const int64_t r = r0 + rr;
            const int p = p0 + pp;
            double a = 0.0;
            if (r < r_end && p < twok) {
                if (p < k) a = to_f64(S[(int64_t)p * ld + r]);
                else a = to_f64(h0[r]) * to_f64(Y[(int64_t)(p - k) * ld + r]);
            }
            As[rr][pp] = a;
        }
        for (int e = tid; e < G1_TR * G1_TC; e += 256) {
            const int rr = e % G1_TR, jj = e / G1_TR;
            const int64_t r = r0 + rr;
            const int j = j0 + jj;
            Bs[rr][jj] = (r < r_end && j < c) ? to_f64(V[(int64_t)j * n + r]) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < G1_TR; ++rr) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = As[rr][ty * 4 + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) b[u] = Bs[rr][tx * 4 + u];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
    double* dst = part + (int64_t)chunk * twok * c;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int p = p0 + ty * 4 + u;
        if (p >= twok) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tx * 4 + v;
            if (j < c) dst[(int64_t)j * twok + p] = acc[u][v];
        }
    }
}

// Z(:, j) = sum over chunks, in chunk order.  Z is column-major 2k x c.
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

__global__ void __launch_bounds__(256) small_solve_blocks(int k, int kmax, int c, const double* __restrict__ Rm,
                                                          const double* __restrict__ Rinv,
                                                          const double* __restrict__ RinvT,
                                                          const double* __restrict__ YHY, const double* __restrict__ Z,
                                                          double* __restrict__ P, double* __restrict__ T,
                                                          int32_t* __restrict__ status) {
    __shared__ double a_sh[256][SB_COLS + 1];
    __shared__ double b_sh[256][SB_COLS + 1];
    const int i = threadIdx.x;
    const int j0 = blockIdx.x * SB_COLS;
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
}

constexpr int G2_TR = 64;   // output rows per tile
constexpr int G2_TC = 64;   // output columns per tile
constexpr int G2_TI = 16;   // pair index per LDS stage

template <typename Ts, typename Th, typename Tv, typename To>
__global__ void __launch_bounds__(256) gemm2_generic(int64_t n, int64_t ld, int k, int c, const Ts* __restrict__ S,
                                                     const Ts* __restrict__ Y, const Th* __restrict__ h0,
                                                     const Tv* __restrict__ V, const double* __restrict__ P,
                                                     const double* __restrict__ T, To* __restrict__ out, int diff) {
    __shared__ double Ss[G2_TI][G2_TR + 2];
    __shared__ double Ys[G2_TI][G2_TR + 2];
    __shared__ double Ts_[G2_TI][G2_TC + 2];
    __shared__ double Ps[G2_TI][G2_TC + 2];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;   // tx: 4 rows each, ty: 4 columns each
    const int64_t r0 = (int64_t)blockIdx.y * G2_TR;
    const int j0 = blockIdx.x * G2_TC;
    double st[4][4] = {}, yp[4][4] = {};
    for (int i0 = 0; i0 < k; i0 += G2_TI) {
        for (int e = tid; e < G2_TI * G2_TR; e += 256) {
            const int rr = e % G2_TR, ii = e / G2_TR;
            const int64_t r = r0 + rr;
            const int i = i0 + ii;
            const bool ok = r < n && i < k;
            Ss[ii][rr] = ok ? to_f64(S[(int64_t)i * ld + r]) : 0.0;
            Ys[ii][rr] = ok ? to_f64(Y[(int64_t)i * ld + r]) : 0.0;
        }
        for (int e = tid; e < G2_TI * G2_TC; e += 256) {
            const int ii = e % G2_TI, jj = e / G2_TI;
            const int i = i0 + ii, j = j0 + jj;
            const bool ok = i < k && j < c;
            Ts_[ii][jj] = ok ? T[(int64_t)j * k + i] : 0.0;
            Ps[ii][jj] = ok ? P[(int64_t)j * k + i] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int ii = 0; ii < G2_TI; ++ii) {
            double s[4], y[4], t[4], p[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                s[u] = Ss[ii][tx * 4 + u];
                y[u] = Ys[ii][tx * 4 + u];
                t[u] = Ts_[ii][ty * 4 + u];
                p[u] = Ps[ii][ty * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    st[u][v] = fma(s[u], t[v], st[u][v]);
                    yp[u][v] = fma(y[u], p[v], yp[u][v]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int j = j0 + ty * 4 + v;
        if (j >= c) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t r = r0 + tx * 4 + u;
            if (r >= n) continue;
            const double hr = to_f64(h0[r]);
            double o = st[u][v] - hr * yp[u][v];
            if (!diff) o += hr * to_f64(V[(int64_t)j * n + r]);
            out[(int64_t)j * n + r] = (To)o;
        }
    }
}

template <typename Th, typename Tv, typename To>
__global__ void scale_by_h0(int64_t n, int c, const Th* __restrict__ h0, const Tv* __restrict__ V,
                            To* __restrict__ out, int diff) {
    const int64_t total = n * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % n;
        out[e] = diff ? (To)0 : (To)(to_f64(h0[r]) * to_f64(V[e]));
    }
}

template <typename Ts, typename Th, typename To>
int apply_generic(bfgsuq_ctx* h, const void* Vv, int c, void* outv, bool diff) {
    const int64_t n = h->n;
    const int k = h->k;
    const Th* h0 = (const Th*)h->h0;
    const Ts* V = (const Ts*)Vv;
    To* out = (To*)outv;
    if (k == 0) {
        int64_t g = std::min<int64_t>(4096, (n * c + 255) / 256);
        hipLaunchKernelGGL((scale_by_h0<Th, Ts, To>), dim3((int)g), dim3(256), 0, h->stream, n, c, h0, V, out,
                           diff ? 1 : 0);
        return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
    }
    const int twok = 2 * k;
    const int ptiles = ceil_div(twok, G1_TP), ctiles = ceil_div(c, G1_TC);
    const int64_t max_chunks = std::max<int64_t>(1, (n + G1_TR - 1) / G1_TR);
    int nchunks = (int)std::min<int64_t>(max_chunks, std::max(1, 2048 / (ptiles * ctiles)));
    const int64_t rows_per_chunk = round_up((n + nchunks - 1) / nchunks, G1_TR);
    nchunks = (int)((n + rows_per_chunk - 1) / rows_per_chunk);
    int rc;
    if ((rc = ensure_ws(h->part, (size_t)nchunks * twok * c * 8)) != BFGS_OK) return rc;
    if ((rc = ensure_ws(h->Z, (size_t)twok * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
    if ((rc = ensure_ws(h->PT, (size_t)2 * h->kmax * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
    double* part = (double*)h->part.ptr;
    double* Z = (double*)h->Z.ptr;
    double* P = (double*)h->PT.ptr;
    double* T = P + (size_t)k * c;
    prof_begin(h, diff ? "hdiff_gemm1" : "apply_gemm1");
    hipLaunchKernelGGL((gemm1_generic<Ts, Th, Ts>), dim3(ptiles, ctiles, nchunks), dim3(256), 0, h->stream, n, h->ld,
                       k, c, (const Ts*)h->S, (const Ts*)h->Y, h0, V, part, rows_per_chunk);
    const int64_t count = (int64_t)twok * c;
    prof_end(h);
    prof_begin(h, "apply_reduce");
    hipLaunchKernelGGL(reduce_partials, dim3(ceil_div(count, 256)), dim3(256), 0, h->stream, count, nchunks, part, Z);
    prof_end(h);
    if (int rc2 = apply_small_solve(h, c, Z, P, T)) return rc2;
    prof_begin(h, diff ? "hdiff_gemm2" : "apply_gemm2");
    hipLaunchKernelGGL((gemm2_generic<Ts, Th, Ts, To>), dim3(ceil_div(c, G2_TC), ceil_div(n, G2_TR)), dim3(256), 0,
                       h->stream, n, h->ld, k, c, (const Ts*)h->S, (const Ts*)h->Y, h0, V, P, T, out,
                       diff ? 1 : 0);
    prof_end(h);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

}  // namespace

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

int apply_block(bfgsuq_ctx* h, const void* V, int32_t ncols, void* out, bool diff) {
    if (mfma_apply_supported(h, ncols)) return mfma_apply(h, V, ncols, out, diff);
    switch (h->storage) {
        case BFGS_F64: return apply_generic<double, double, double>(h, V, ncols, out, diff);
        case BFGS_F32: return apply_generic<float, float, float>(h, V, ncols, out, diff);
        case BFGS_BF16: return apply_generic<bf16_t, float, float>(h, V, ncols, out, diff);
    }
    return BFGS_ERR_ARG;
}
