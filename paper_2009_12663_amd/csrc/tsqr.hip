// Blocked Householder TSQR of E (n x c, column-major, c <= 256) for Alg. 3's
// "E = Q R": Q explicit (n x c, column-major), R upper triangular (c x c, row-major).
//
// Layout.  E is split into `nchains` contiguous row ranges, one workgroup each.
// A workgroup keeps an upper-triangular c x c slot (packed, LDS) and folds its
// rows in, BT rows at a time.  The BT x c tile lives in registers as 16 x 16
// float64 matrix-core accumulator fragments: wave w owns column tile w (columns
// 16w .. 16w + 15), lane l holds rows 16 rt + l/16 + 4 r of column 16 w + l%16.
//
// Leaves (forward).  One quad of lanes per column folds each tile with one
// barrier per reflector (leaf_forward_q); the reflectors are stored in the panel
// layout below, with each panel's T formed from them while they are in registers.
//
// Tree fold (forward).  Panel p (column tile p) is factored by its owner
// wave, one Householder reflector per column acting on (slot row j, tile rows);
// the panel's reflectors form the compact WY block I - V T V^T (V: tile part,
// the slot part of reflector j is the unit vector e_j; T upper triangular).  The
// waves right of the panel then apply its transpose to their columns on the
// matrix cores:  W = S_p + V^T A,  W' = T^T W,  S_p -= W',  A -= V W', where S_p
// is the panel's 16 slot rows.  Panels and T alternate between two LDS buffers,
// so panel p+1 is factored while the other waves still apply panel p.
// The slot starts at zero, so a column's first non-zero tile swaps into the slot
// (tau = 1) and the slot rows carry no part of Q.
//
// Q (backward).  The per-chain R factors are combined by a binary tree with the
// same fold (reading the second R as tile rows).  Q is then formed by applying the
// stored blocks in reverse to the identity at the root and to zero tile rows at
// the leaves: W = S_p + V^T A,  W' = T W,  S_p -= W',  A -= V W'.  Every slot met
// on the way stays upper triangular.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace {

constexpr int PW = 16;           // panel width = column tile width
constexpr int TS_LD = PW + 1;    // T and G row pitch in LDS

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int tri_index(int j, int col, int c) {
    // packed upper triangle, row-major: row j holds columns j..c-1
    return j * c - (j * (j - 1)) / 2 + (col - j);
}

// 1 / sqrt(t) for t > 0, denormal t included (hardware estimate refined by two
// Newton steps).
__device__ __forceinline__ double rsqrt_nr(double t) {
    double y = __builtin_amdgcn_rsq(t);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double ty = t * y;
        const double e = fma(-ty, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// 1 / x for normal x (hardware estimate refined by two Newton steps).
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

// x + x(lane ^ 16) + x(lane ^ 32) + x(lane ^ 48): the sum over the four 16-lane rows
// that share lane % 16.  v_permlane{16,32}_swap with both operands equal to x
// returns, across its two results, each lane's own value and its partner's.
__device__ __forceinline__ double add_perm16(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    const double a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
    const double b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
    return a + b;
}

__device__ __forceinline__ double add_perm32(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    const double a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
    const double b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
    return a + b;
}

__device__ __forceinline__ double row_sum4(double x) { return add_perm32(add_perm16(x)); }

__device__ __forceinline__ double read_lane(double x, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// x of lane src (any lane, chosen per lane)
__device__ __forceinline__ double bpermute_f64(double x, int src) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)u);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// LDS: Vp[2][PW][VLD] | Ts[2][PW][TS_LD] | Gs[PW][TS_LD] | tau[PW] | slot
template <int BT>
struct Layout {
    static constexpr int RT = BT / 16;
    static constexpr int VLD = BT + 2;
    static constexpr int VP = PW * VLD;            // doubles per panel buffer
    static constexpr int TSZ = PW * TS_LD;
    static constexpr int HEAD = 2 * VP + 2 * TSZ + TSZ + PW;
    static constexpr int PS = PW * BT + PW * PW;   // doubles per stored panel (V then T)
};

template <int BT, typename SlotT>
size_t lds_bytes(int c) {
    return (size_t)Layout<BT>::HEAD * sizeof(double) + (size_t)c * (c + 1) / 2 * sizeof(SlotT);
}

// Factor panel p (owner wave): 16 reflectors on (slot rows 16p.., tile columns).
// Leaves V in Vp ([refl][row]), T in Ts, copies both to `store` (V: [refl][BT], then T).
template <int BT, typename SlotT>
__device__ void factor_panel(SlotT* slot, v4d (&A)[Layout<BT>::RT], int c, int p, double* Vp, double* Ts,
                             double* Gs, double* tau_s, double* store) {
    constexpr int RT = Layout<BT>::RT, VLD = Layout<BT>::VLD;
    const int lane = threadIdx.x & 63, jl = lane & 15, q = lane >> 4;
    const int j0 = p * PW, col = j0 + jl;
    __builtin_amdgcn_s_setprio(3);   // the panel is the critical path
    for (int jj = 0; jj < PW; ++jj) {
        const int j = j0 + jj;
        // slot(j, j) and slot(j, col): no earlier reflector of this panel touches row j
        const int dj = j < c ? tri_index(j, j, c) : 0;
        const bool mine = jl > jj && col < c;
        const int ij = mine ? tri_index(j, col, c) : 0;
        const double rjj_pre = (double)slot[dj];
        const double rr_pre = mine ? (double)slot[ij] : 0.0;
        // norm^2 of column jj's tile part (every lane computes its own column's);
        // four independent partial sums keep the FMA chains short
        double pp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) pp[r] = fma(A[rt][r], A[rt][r], pp[r]);
        const double part = row_sum4((pp[0] + pp[1]) + (pp[2] + pp[3]));
        const double xn2 = read_lane(part, jj);
        double tau = 0.0, beta = 0.0, sc = 0.0;
        if (j < c && xn2 > 0.0) {
            // beta = -sign(rjj) |(rjj, x)|, tau = (beta - rjj) / beta, v = x / (rjj - beta);
            // |beta| and |rjj - beta| are >= sqrt(xn2) >= 2^-537: both reciprocals are of
            // normal numbers (their product need not be)
            const double rjj = rjj_pre;
            const double t = fma(rjj, rjj, xn2);
            beta = -copysign(t * rsqrt_nr(t), rjj);
            const double u = rjj - beta;
            tau = -u * rcp_nr(beta);
            sc = rcp_nr(u);
        }
        if (jl == jj) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    A[rt][r] *= sc;
                    Vp[jj * VLD + rt * 16 + q + 4 * r] = A[rt][r];
                }
        }
        if (lane == 0) {
            if (tau != 0.0) slot[dj] = (SlotT)beta;
            tau_s[jj] = tau;
        }
        wave_sync();
        if (tau != 0.0) {
            double dp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) dp[r] = fma(Vp[jj * VLD + rt * 16 + q + 4 * r], A[rt][r], dp[r]);
            const double d = row_sum4((dp[0] + dp[1]) + (dp[2] + dp[3]));
            if (mine) {
                const double rr = rr_pre;
                const double w = (rr + d) * tau;
                if (q == 0) slot[ij] = (SlotT)(rr - w);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) A[rt][r] = fma(-w, Vp[jj * VLD + rt * 16 + q + 4 * r], A[rt][r]);
            }
        }
        wave_sync();
    }
    __builtin_amdgcn_s_setprio(0);
    // G = V^T V (tile parts; the slot parts are distinct unit vectors) on the matrix core
    v4d g = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < BT / 4; ++ks) {
        const double a = Vp[jl * VLD + ks * 4 + q];
        g = mfma64(a, a, g);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Gs[(q + 4 * r) * TS_LD + jl] = g[r];
    wave_sync();
    // T(a, i) = -tau_i sum_{a <= b < i} T(a, b) G(b, i), T(a, a) = tau_a: row a of T
    // depends only on row a, so lane a builds it alone, in registers.
    if (lane < PW) {
        double trow[PW];
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            double sacc = 0.0;
#pragma unroll
            for (int b = 0; b < i; ++b) sacc = fma(trow[b], Gs[b * TS_LD + i], sacc);
            const double ti = tau_s[i];
            trow[i] = i < lane ? 0.0 : (i == lane ? ti : -ti * sacc);
        }
#pragma unroll
        for (int i = 0; i < PW; ++i) Ts[lane * TS_LD + i] = trow[i];
    }
    // copy V and T out for the backward pass (coalesced)
    for (int e = lane; e < PW * BT; e += 64) store[e] = Vp[(e / BT) * VLD + e % BT];
    for (int e = lane; e < PW * PW; e += 64) store[PW * BT + e] = Ts[(e / PW) * TS_LD + e % PW];
    wave_sync();
}

// Apply panel p's block to this wave's column tile w:
//   W = S_p + V^T A;  W' = op(T) W (op = transpose in the fold);  S_p -= W';  A -= V W'.
template <int BT, typename SlotT, bool TRANS>
__device__ __forceinline__ void apply_panel(SlotT* slot, v4d (&A)[Layout<BT>::RT], int c, int p, int w,
                                            const double* Vp, const double* Ts) {
    constexpr int RT = Layout<BT>::RT, VLD = Layout<BT>::VLD;
    const int lane = threadIdx.x & 63, jl = lane & 15, q = lane >> 4;
    const int r0 = p * PW, col = w * PW + jl;
    v4d W;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = r0 + q + 4 * r;
        W[r] = (col < c && row <= col) ? (double)slot[tri_index(row, col, c)] : 0.0;
    }
#pragma unroll
    for (int ks = 0; ks < BT / 4; ++ks) W = mfma64(Vp[jl * VLD + ks * 4 + q], A[ks >> 2][ks & 3], W);
    v4d Wp = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const double a = TRANS ? Ts[(ks * 4 + q) * TS_LD + jl] : Ts[jl * TS_LD + ks * 4 + q];
        Wp = mfma64(a, W[ks], Wp);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = r0 + q + 4 * r;
        if (col < c && row <= col) {
            const int idx = tri_index(row, col, c);
            slot[idx] = (SlotT)((double)slot[idx] - Wp[r]);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) A[rt] = mfma64(-Vp[(ks * 4 + q) * VLD + rt * 16 + jl], Wp[ks], A[rt]);
}

template <typename SlotT>
__device__ void slot_zero(SlotT* slot, int c) {
    const int tri = c * (c + 1) / 2;
    for (int e = threadIdx.x; e < tri; e += blockDim.x) slot[e] = (SlotT)0;
    __syncthreads();
}

template <typename SlotT>
__device__ void slot_load(SlotT* slot, const double* M, int c) {
    for (int j = 0; j < c; ++j)
        for (int col = j + threadIdx.x; col < c; col += blockDim.x) slot[tri_index(j, col, c)] = (SlotT)M[(int64_t)j * c + col];
    __syncthreads();
}

template <typename SlotT>
__device__ void slot_store(const SlotT* slot, double* M, int c) {
    for (int j = 0; j < c; ++j)
        for (int col = threadIdx.x; col < c; col += blockDim.x)
            M[(int64_t)j * c + col] = col >= j ? (double)slot[tri_index(j, col, c)] : 0.0;
    __syncthreads();
}

// Fold the tile in A into the slot, panels p0 .. np-1; panel p's V and T go to
// store + p * PS.
template <int BT, typename SlotT>
__device__ void fold_tile(SlotT* slot, v4d (&A)[Layout<BT>::RT], int c, int p0, double* lds, double* store) {
    constexpr int VP = Layout<BT>::VP, TSZ = Layout<BT>::TSZ, PS = Layout<BT>::PS;
    const int wave = threadIdx.x >> 6;
    const int np = (c + PW - 1) / PW;
    double* Vbuf = lds;
    double* Tbuf = lds + 2 * VP;
    double* Gs = Tbuf + 2 * TSZ;
    double* tau_s = Gs + TSZ;
    for (int p = p0; p < np; ++p) {
        const int b = (p - p0) & 1;
        if (wave == p) factor_panel<BT, SlotT>(slot, A, c, p, Vbuf + b * VP, Tbuf + b * TSZ, Gs, tau_s, store + (int64_t)p * PS);
        __syncthreads();
        if (wave > p) apply_panel<BT, SlotT, true>(slot, A, c, p, wave, Vbuf + b * VP, Tbuf + b * TSZ);
    }
    __syncthreads();
}

// Apply the stored panels np-1 .. p0 (backward) to (slot, A).  Each panel's V and T
// are staged through LDS (two buffers); the global loads run two panels ahead of the
// panel being applied, in two register sets of PF doubles per thread.  When PF values
// per thread cannot hold a panel (few columns, so few threads), a panel is copied
// straight to LDS instead.
template <int BT, typename SlotT, int PF>
__device__ void unfold_tile(SlotT* slot, v4d (&A)[Layout<BT>::RT], int c, int p0, double* lds, const double* store) {
    constexpr int VLD = Layout<BT>::VLD, VP = Layout<BT>::VP, TSZ = Layout<BT>::TSZ, PS = Layout<BT>::PS;
    const int wave = threadIdx.x >> 6;
    const int np = (c + PW - 1) / PW;
    double* Vbuf = lds;
    double* Tbuf = lds + 2 * VP;
    const int nthr = blockDim.x;
    const bool staged = PF * nthr >= PS;
    auto ld = [&](int P, double (&pre)[PF]) {
        const double* src = store + (int64_t)P * PS;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int e = threadIdx.x + k * nthr;
            pre[k] = e < PS ? src[e] : 0.0;
        }
    };
    auto st = [&](int B, const double (&pre)[PF]) {
        double* v = Vbuf + B * VP;
        double* t = Tbuf + B * TSZ;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int e = threadIdx.x + k * nthr;
            if (e < PW * BT) v[(e / BT) * VLD + e % BT] = pre[k];
            else if (e < PS) t[((e - PW * BT) / PW) * TS_LD + (e - PW * BT) % PW] = pre[k];
        }
    };
    auto copy = [&](int P, int B) {
        for (int e = threadIdx.x; e < PS; e += nthr) {
            const double x = store[(int64_t)P * PS + e];
            if (e < PW * BT) Vbuf[B * VP + (e / BT) * VLD + e % BT] = x;
            else Tbuf[B * TSZ + ((e - PW * BT) / PW) * TS_LD + (e - PW * BT) % PW] = x;
        }
    };
    double pa[PF], pb[PF];
    __syncthreads();
    if (staged) {
        ld(np - 1, pa);
        st(0, pa);
        if (np - 2 >= p0) ld(np - 2, pb);
    } else {
        copy(np - 1, 0);
    }
    __syncthreads();
    // panel p from buffer b; x holds panel p - 1 (loaded two panels ago), y receives p - 2
    auto step = [&](int p, int b, double (&x)[PF], double (&y)[PF]) {
        if (staged && p - 2 >= p0) ld(p - 2, y);
        if (wave >= p) apply_panel<BT, SlotT, false>(slot, A, c, p, wave, Vbuf + b * VP, Tbuf + b * TSZ);
        if (p - 1 >= p0) {
            if (staged) st(b ^ 1, x);
            else copy(p - 1, b ^ 1);
        }
        __syncthreads();
    };
    // panel np - 1 - 2i uses buffer 0, the one after it buffer 1
    for (int p = np - 1; p >= p0; p -= 2) {
        step(p, 0, pb, pa);
        if (p - 1 < p0) break;
        step(p - 1, 1, pa, pb);
    }
}

// ---------------------------------------------------------------------------
// Leaf fold with a quad of lanes per column (one barrier per reflector).  The
// leaves' critical path is the chain of c reflectors per tile; handing each column
// to its own quad (16 rows per lane, quad DPP reductions) and building reflector
// j+1 in the quad of column j+1 right after it applies reflector j keeps that
// chain shorter than the per-wave panel factorisation.  The reflectors and each
// panel's T are written in the panel layout of the blocked backward pass.
// ---------------------------------------------------------------------------
constexpr int QT = 64;                 // tile rows (matches the blocked pass's BT = 64)
constexpr int LPC = 4;                 // lanes per column
constexpr int RPL = QT / LPC;          // rows per lane: row t = i * LPC + g

template <int CTRL>
__device__ __forceinline__ double quad_perm(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double quad_sum(double x) {
    x += quad_perm<0xB1>(x);   // lanes (1,0,3,2)
    x += quad_perm<0x4E>(x);   // lanes (2,3,0,1)
    return x;
}

// Reflector j from (slot[j][j], tile column j held by this quad): the tile part
// overwrites a[], goes to vbuf; tau to tau_sh and taus_lds[j].
template <typename SlotT>
__device__ __forceinline__ void q_make_reflector(SlotT* slot, double (&a)[RPL], int c, int j, int g, double* vbuf,
                                                 double* tau_sh, double* taus_lds) {
    double p4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < RPL; ++i) p4[i & 3] = fma(a[i], a[i], p4[i & 3]);
    const double xn2 = quad_sum((p4[0] + p4[1]) + (p4[2] + p4[3]));
    const int dj = tri_index(j, j, c);
    const double rjj = (double)slot[dj];
    double tau = 0.0;
    if (xn2 > 0.0) {
        // as in factor_panel: two reciprocals of normal-range numbers
        const double t = fma(rjj, rjj, xn2);
        const double beta = -copysign(t * rsqrt_nr(t), rjj);
        const double u = rjj - beta;
        tau = -u * rcp_nr(beta);
        const double sc = rcp_nr(u);
#pragma unroll
        for (int i = 0; i < RPL; ++i) a[i] *= sc;
        if (g == 0) slot[dj] = (SlotT)beta;
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) vbuf[i * LPC + g] = a[i];
    if (g == 0) {
        *tau_sh = tau;
        taus_lds[j] = tau;
    }
}

template <typename SlotT>
__device__ __forceinline__ void q_reflect_column(SlotT* slot, double (&a)[RPL], int c, int j, int col, int g,
                                                 const double* v, double tau) {
    double p4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < RPL; ++i) p4[i & 3] = fma(v[i * LPC + g], a[i], p4[i & 3]);
    const double s = quad_sum((p4[0] + p4[1]) + (p4[2] + p4[3]));
    const int idx = tri_index(j, col, c);
    const double r = (double)slot[idx];
    const double w = (r + s) * tau;
    if (g == 0) slot[idx] = (SlotT)(r - w);
#pragma unroll
    for (int i = 0; i < RPL; ++i) a[i] = fma(-w, v[i * LPC + g], a[i]);
}

// LDS of the quad fold: vbuf[2][QT] | tau_sh[2] | taus_lds[256] | slot
constexpr int QF_HEAD = 2 * QT + 2 + 256;

template <typename SlotT>
size_t qf_lds_bytes(int c) {
    return (size_t)QF_HEAD * sizeof(double) + (size_t)c * (c + 1) / 2 * sizeof(SlotT);
}

template <typename TE, typename SlotT>
__global__ void __launch_bounds__(1024) leaf_forward_q(int64_t n, int c, int64_t rows_per_chain,
                                                       const TE* __restrict__ E, double* __restrict__ refl,
                                                       double* __restrict__ Rs) {
    extern __shared__ double lds[];
    double* vbuf = lds;
    double* tau_sh = vbuf + 2 * QT;
    double* taus_lds = tau_sh + 2;
    SlotT* slot = (SlotT*)(lds + QF_HEAD);
    constexpr int PS = Layout<QT>::PS;
    const int ch = blockIdx.x, col = threadIdx.x / LPC, g = threadIdx.x % LPC;
    const int np = (c + PW - 1) / PW;
    const int64_t r_begin = ch * rows_per_chain;
    const int64_t r_end = min(n, r_begin + rows_per_chain);
    const int tiles_per_chain = (int)(rows_per_chain / QT);
    slot_zero(slot, c);
    for (int tile = 0; r_begin + (int64_t)tile * QT < r_end; ++tile) {
        const int64_t r0 = r_begin + (int64_t)tile * QT;
        double a[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int64_t r = r0 + i * LPC + g;
            a[i] = (col < c && r < r_end) ? to_f64(E[(int64_t)col * n + r]) : 0.0;
        }
        if (col == 0) q_make_reflector(slot, a, c, 0, g, vbuf, tau_sh, taus_lds);
        __syncthreads();
        for (int j = 0; j < c; ++j) {
            const int buf = j & 1;
            const double tau = tau_sh[buf];
            if (col > j && col < c && tau != 0.0) q_reflect_column(slot, a, c, j, col, g, vbuf + buf * QT, tau);
            if (col == j + 1 && j + 1 < c)
                q_make_reflector(slot, a, c, j + 1, g, vbuf + (buf ^ 1) * QT, tau_sh + (buf ^ 1), taus_lds);
            __syncthreads();
        }
        // reflector col: tile part (rows t = i * LPC + g) in the panel layout
        const int64_t gtile = (int64_t)ch * tiles_per_chain + tile;
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;   // wave = panel
        double* dst = refl + (gtile * np + wave) * PS;
#pragma unroll
        for (int i = 0; i < RPL; ++i) dst[(col % PW) * QT + i * LPC + g] = a[i];
        // The panel's compact-WY factor T (I - V T V^T, T upper triangular) from the
        // reflectors still in registers.  G = V^T V on the matrix cores: V's rows
        // 4 ks .. 4 ks + 3 sit in a[ks] of the quads, one lane permutation away from the
        // A/B operand layout.  Then T column by column: lane r < 16 keeps row r, and
        // G(b, i) (accumulator element b / 4 of lane 16 (b % 4) + i) is broadcast.
        {
            const int src = 4 * (lane & 15) + (lane >> 4);
            v4d gacc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < RPL; ++ks) {
                const double v = bpermute_f64(a[ks], src);
                gacc = mfma64(v, v, gacc);
            }
            const int r = lane & 15;
            double trow[PW];
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const int ci = wave * PW + i;
                const double tau_i = ci < c ? taus_lds[ci] : 0.0;
                double sacc = 0.0;
#pragma unroll
                for (int b = 0; b < i; ++b) sacc = fma(trow[b], read_lane(gacc[b / 4], 16 * (b % 4) + i), sacc);
                trow[i] = i < r ? 0.0 : (i == r ? tau_i : -tau_i * sacc);
            }
            if (lane < PW) {
#pragma unroll
                for (int i = 0; i < PW; ++i) dst[PW * QT + lane * PW + i] = trow[i];
            }
        }
    }
    slot_store(slot, Rs + (int64_t)ch * c * c, c);
}

// ---------------------------------------------------------------------------
// Kernels of the blocked passes.  Leaf tile g of chain ch stores its panels at
// refl + (g * np + p) * PS.
// ---------------------------------------------------------------------------
template <typename TQ, typename SlotT, int BT, int PF>
__global__ void __launch_bounds__(1024) leaf_backward(int64_t n, int c, int64_t rows_per_chain,
                                                      const double* __restrict__ refl, const double* __restrict__ Qtop,
                                                      TQ* __restrict__ Q) {
    extern __shared__ double lds[];
    constexpr int RT = Layout<BT>::RT, PS = Layout<BT>::PS;
    SlotT* slot = (SlotT*)(lds + Layout<BT>::HEAD);
    const int ch = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, jl = lane & 15, q = lane >> 4;
    const int np = (c + PW - 1) / PW;
    const int col = wave * PW + jl;
    const int64_t r_begin = ch * rows_per_chain;
    if (r_begin >= n) return;   // uniform: whole workgroup leaves
    const int64_t r_end = min(n, r_begin + rows_per_chain);
    const int tiles_per_chain = (int)(rows_per_chain / BT);
    const int ntiles = (int)((r_end - r_begin + BT - 1) / BT);
    slot_load(slot, Qtop + (int64_t)ch * c * c, c);
    for (int tile = ntiles - 1; tile >= 0; --tile) {
        const int64_t r0 = r_begin + (int64_t)tile * BT;
        const int64_t gtile = (int64_t)ch * tiles_per_chain + tile;
        v4d A[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) A[rt] = v4d{0, 0, 0, 0};
        unfold_tile<BT, SlotT, PF>(slot, A, c, 0, lds, refl + gtile * np * PS);
        if (col < c) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = r0 + rt * 16 + q + 4 * r;
                    if (row < r_end) Q[(int64_t)col * n + row] = (TQ)A[rt][r];
                }
        }
    }
}

// Tree: combine i of a level merges chain a = i * 2 * stride with b = a + stride;
// its tile t (rows t * BT .. of R_b) stores panels at tree + ((comb_off + i) * ntt + t) * np * PS.
template <typename SlotT, int BT>
__global__ void __launch_bounds__(1024) tree_forward(int c, int stride, int64_t comb_off, double* __restrict__ Rs,
                                                     double* __restrict__ tree) {
    extern __shared__ double lds[];
    constexpr int RT = Layout<BT>::RT, PS = Layout<BT>::PS;
    SlotT* slot = (SlotT*)(lds + Layout<BT>::HEAD);
    const int i = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, jl = lane & 15, q = lane >> 4;
    const int np = (c + PW - 1) / PW, ntt = (c + BT - 1) / BT;
    const int col = wave * PW + jl;
    const int a_idx = i * 2 * stride, b_idx = a_idx + stride;
    const double* Rb = Rs + (int64_t)b_idx * c * c;
    slot_load(slot, Rs + (int64_t)a_idx * c * c, c);
    for (int t = 0; t < ntt; ++t) {
        v4d A[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = t * BT + rt * 16 + q + 4 * r;
                A[rt][r] = (col < c && row < c && col >= row) ? Rb[(int64_t)row * c + col] : 0.0;
            }
        fold_tile<BT, SlotT>(slot, A, c, (t * BT) / PW, lds, tree + ((comb_off + i) * ntt + t) * np * PS);
    }
    slot_store(slot, Rs + (int64_t)a_idx * c * c, c);
}

template <typename SlotT, int BT, int PF>
__global__ void __launch_bounds__(1024) tree_backward(int c, int stride, int64_t comb_off, double* __restrict__ Qtop,
                                                      const double* __restrict__ tree) {
    extern __shared__ double lds[];
    constexpr int RT = Layout<BT>::RT, PS = Layout<BT>::PS;
    SlotT* slot = (SlotT*)(lds + Layout<BT>::HEAD);
    const int i = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, jl = lane & 15, q = lane >> 4;
    const int np = (c + PW - 1) / PW, ntt = (c + BT - 1) / BT;
    const int col = wave * PW + jl;
    const int a_idx = i * 2 * stride, b_idx = a_idx + stride;
    double* Qb = Qtop + (int64_t)b_idx * c * c;
    slot_load(slot, Qtop + (int64_t)a_idx * c * c, c);
    for (int t = ntt - 1; t >= 0; --t) {
        v4d A[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) A[rt] = v4d{0, 0, 0, 0};
        unfold_tile<BT, SlotT, PF>(slot, A, c, (t * BT) / PW, lds, tree + ((comb_off + i) * ntt + t) * np * PS);
        if (col < c) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = t * BT + rt * 16 + q + 4 * r;
                    if (row < c) Qb[(int64_t)row * c + col] = A[rt][r];
                }
        }
    }
    slot_store(slot, Qtop + (int64_t)a_idx * c * c, c);
}

__global__ void set_identity_kernel(double* __restrict__ M, int c) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c * c; e += gridDim.x * blockDim.x)
        M[e] = (e / c == e % c) ? 1.0 : 0.0;
}

inline int floor_pow2(int64_t x) {
    int p = 1;
    while ((int64_t)p * 2 <= x) p *= 2;
    return p;
}

// PF: doubles per thread that stage one stored panel in the backward passes.
template <typename TO, typename SlotT, int BT, int PF>
int tsqr_impl(bfgsuq_ctx* h, int c, const TO* E, TO* Q, double** R_out) {
    constexpr int PS = Layout<BT>::PS;
    const int64_t n = h->n;
    const int np = (c + PW - 1) / PW;
    const int threads = 64 * np;
    const int64_t tiles_total = (n + BT - 1) / BT;
    const int nchains = (int)std::min<int64_t>(h->qr_chains, floor_pow2(std::max<int64_t>(1, tiles_total / 2)));
    const int64_t rows_per_chain = round_up((n + nchains - 1) / nchains, BT);
    const int tiles_per_chain = (int)(rows_per_chain / BT);
    const int ntt = (c + BT - 1) / BT;
    int rc;
    const size_t leaf_doubles = (size_t)nchains * tiles_per_chain * np * PS;
    const size_t tree_doubles = (size_t)std::max(1, nchains - 1) * ntt * np * PS;
    if ((rc = ensure_ws(h->refl, (leaf_doubles + tree_doubles) * 8)) != BFGS_OK) return rc;
    if ((rc = ensure_ws(h->Rtree, (size_t)2 * nchains * c * c * 8)) != BFGS_OK) return rc;
    double* refl = (double*)h->refl.ptr;
    double* tree = refl + leaf_doubles;
    double* Rs = (double*)h->Rtree.ptr;
    double* Qtop = Rs + (size_t)nchains * c * c;
    const size_t smem = lds_bytes<BT, SlotT>(c);
    // Raise the dynamic-LDS limit once per instantiation (never while a graph is being captured).
    static bool attr_done = false;
    if (!attr_done) {
        const int lim = 160 * 1024;
        if (hipFuncSetAttribute((const void*)leaf_backward<TO, SlotT, BT, PF>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
            hipFuncSetAttribute((const void*)tree_forward<SlotT, BT>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
            hipFuncSetAttribute((const void*)tree_backward<SlotT, BT, PF>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
            return BFGS_ERR_HIP;
        attr_done = true;
    }
    static bool attr_q = false;
    if (!attr_q) {
        if (hipFuncSetAttribute((const void*)leaf_forward_q<TO, SlotT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024) != hipSuccess)
            return BFGS_ERR_HIP;
        attr_q = true;
    }
    prof_begin(h, "tsqr_leaf_fwd");
    hipLaunchKernelGGL((leaf_forward_q<TO, SlotT>), dim3(nchains), dim3(LPC * 16 * np), qf_lds_bytes<SlotT>(c),
                       h->stream, n, c, rows_per_chain, E, refl, Rs);
    prof_end(h);
    prof_begin(h, "tsqr_tree");
    int64_t off = 0;
    for (int stride = 1; stride < nchains; stride *= 2) {
        const int ncomb = nchains / (2 * stride);
        hipLaunchKernelGGL((tree_forward<SlotT, BT>), dim3(ncomb), dim3(threads), smem, h->stream, c, stride, off, Rs,
                           tree);
        off += ncomb;
    }
    hipLaunchKernelGGL(set_identity_kernel, dim3(64), dim3(256), 0, h->stream, Qtop, c);
    for (int stride = nchains / 2; stride >= 1; stride /= 2) {
        const int ncomb = nchains / (2 * stride);
        off -= ncomb;
        hipLaunchKernelGGL((tree_backward<SlotT, BT, PF>), dim3(ncomb), dim3(threads), smem, h->stream, c, stride, off,
                           Qtop, tree);
    }
    prof_end(h);
    prof_begin(h, "tsqr_leaf_bwd");
    hipLaunchKernelGGL((leaf_backward<TO, SlotT, BT, PF>), dim3(nchains), dim3(threads), smem, h->stream, n, c,
                       rows_per_chain, refl, Qtop, Q);
    prof_end(h);
    *R_out = Rs;   // chain 0 holds the final R (row-major, upper triangular)
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

template <typename TO>
int tsqr_dispatch(bfgsuq_ctx* h, int c, const TO* E, TO* Q, double** R_out) {
    if (c < 1 || c > 256) return BFGS_ERR_ARG;
    // 64-row tiles keep a tile's fragments, the staging registers and the panel work
    // within 128 registers per lane (1024-thread workgroups); the slot is float64
    // whenever it fits in LDS (c <= 184) and float32 above that
    const size_t lim = 160 * 1024;
    const bool dslot = lds_bytes<64, double>(c) <= lim && qf_lds_bytes<double>(c) <= lim;
    // staging doubles per thread for one stored panel (64 * ceil(c / 16) threads); more
    // than 8 (c <= 32) copies panels straight to LDS
    const int pf = ceil_div(Layout<64>::PS, 64 * ceil_div(c, PW));
    if (pf <= 2) return dslot ? tsqr_impl<TO, double, 64, 2>(h, c, E, Q, R_out) : tsqr_impl<TO, float, 64, 2>(h, c, E, Q, R_out);
    if (pf <= 3) return dslot ? tsqr_impl<TO, double, 64, 3>(h, c, E, Q, R_out) : tsqr_impl<TO, float, 64, 3>(h, c, E, Q, R_out);
    if (pf <= 5) return dslot ? tsqr_impl<TO, double, 64, 5>(h, c, E, Q, R_out) : tsqr_impl<TO, float, 64, 5>(h, c, E, Q, R_out);
    return dslot ? tsqr_impl<TO, double, 64, 8>(h, c, E, Q, R_out) : tsqr_impl<TO, float, 64, 8>(h, c, E, Q, R_out);
}

}  // namespace

int tsqr_run(bfgsuq_ctx* h, int c, const float* E, float* Q, double** R_out) { return tsqr_dispatch(h, c, E, Q, R_out); }
int tsqr_run(bfgsuq_ctx* h, int c, const double* E, double* Q, double** R_out) {
    return tsqr_dispatch(h, c, E, Q, R_out);
}
