// Householder TSQR of E (n x c, column-major, c <= 256) for Alg. 3's "E = Q R":
// Q explicit (n x c, column-major, or chain-blocked: each chain's rows one
// contiguous column-major block), R upper triangular (c x c, row-major).
//
// Layout.  E is split into `nchains` contiguous row ranges, one workgroup each.
// A workgroup keeps an upper-triangular c x c slot (packed, LDS) and folds its
// rows in, 64 at a time.  The slot starts at zero, so a column's first non-zero
// tile swaps into the slot (tau = 1) and the slot rows carry no part of Q.
//
// Forward (leaf_forward_q, tree_forward_q).  One quad of lanes per column holds
// the column's 64 tile rows (16 per lane); reflector j acts on (slot row j, tile
// rows).  Wave k (in the fold's numbering: hardware waves take the groups in the
// order qf_perm gives, which spreads the groups that apply many blocks over the
// SIMDs) owns columns 16 k .. 16 k + 15 and builds their group of 16
// reflectors; there is no workgroup barrier: the groups pass through a ring of LDS
// entries with per-entry ready/done counters (q_fold).  The two waves after a
// builder apply its reflectors one at a time as they are published (they build the
// next groups); waves further right apply the whole group as one compact-WY block
// (I - V T V^T, V the tile parts; the slot part of reflector j is the unit vector
// e_j; T upper triangular) on the float64 matrix cores.  Every group is also stored
// as a panel (V, T) for the backward pass.  The per-chain R factors are combined by
// a binary tree with the same fold, R_b read as tile rows (tile t is zero left of
// column 64 t).
//
// Backward (tree_backward, leaf_backward).  Q is formed by applying the stored
// panels in reverse to the identity at the root and to zero tile rows at the
// leaves, on the float64 matrix cores from register-resident accumulator tiles
// (the wave of group w, as in the forward folds, owns column tile w; lane l holds
// rows 16 rt + l/16 + 4 r of column 16 w + l%16):  W = S_p + V^T A,  W' = T W,  S_p -= W',  A -= V W', with S_p the
// panel's 16 slot rows.  Every slot met on the way stays upper triangular.
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

// 1 / sqrt(t) for t > 0, denormal t included.  The hardware estimate is within
// 2^-24 relative (measured on gfx950); with e = 1 - t y^2 the exact value is
// y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2 / 8 + O(e^3)), so one third-order step
// leaves an error near 2^-72, below the float64 rounding.
__device__ __forceinline__ double rsqrt_nr(double t) {
    const double y = __builtin_amdgcn_rsq(t);
    const double e = fma(-(t * y), y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// 1 / x for normal x: the hardware estimate (within 2^-24 relative) refined by
// one third-order step, y / (1 - e) = y (1 + e + e^2 + O(e^3)) with e = 1 - x y.
__device__ __forceinline__ double rcp_nr(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

__device__ __forceinline__ double read_lane(double x, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The lane index as a value the compiler cannot see through: masks computed from it
// are formed where they are used, instead of being hoisted out of the fold's loops
// into scalar registers (the fold has none to spare, and spilled masks cost more to
// restore than to recompute).
__device__ __forceinline__ int fresh_lane() {
    int l = (int)(threadIdx.x & 63);
    asm volatile("" : "+v"(l));
    return l;
}

// The column group this wave owns: hardware wave w (on SIMD w mod 4) takes group
// (perm >> 4 w) & 15, so that the heavy groups (those with many groups before them)
// are spread over the SIMDs.
__device__ __forceinline__ int qf_group(uint64_t perm) { return (int)((perm >> (4 * (threadIdx.x >> 6))) & 15u); }

// x of lane src (any lane, chosen per lane)
__device__ __forceinline__ double bpermute_f64(double x, int src) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)u);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// LDS of the backward passes: Vp[2][PW][VLD] | Ts[2][PW][TS_LD] | slot
template <int BT>
struct Layout {
    static constexpr int RT = BT / 16;
    static constexpr int VLD = BT + 2;
    static constexpr int VP = PW * VLD;            // doubles per panel buffer
    static constexpr int TSZ = PW * TS_LD;
    static constexpr int HEAD = 2 * VP + 2 * TSZ;
    static constexpr int PS = PW * BT + PW * PW;   // doubles per stored panel (V then T)
};

template <int BT, typename SlotT>
size_t lds_bytes(int c) {
    return (size_t)Layout<BT>::HEAD * sizeof(double) + (size_t)c * (c + 1) / 2 * sizeof(SlotT);
}

// Apply panel p's block to this wave's column tile w:
//   W = S_p + V^T A;  W' = op(T) W (op = transpose for Q^T, identity for Q);  S_p -= W';  A -= V W'.
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

// A c x c upper-triangular matrix (row-major in M) into and out of the packed slot.
// Thread t takes column t (and t + blockDim.x, ...), rows in groups of SL_ROWS whose
// loads are all in flight before the first is stored: one row at a time would wait a
// full memory round trip per row.  Loads past the diagonal are clamped to it (issued,
// unused), so that none is conditional.
constexpr int SL_ROWS = 16;

template <typename SlotT>
__device__ void slot_load(SlotT* slot, const double* M, int c) {
    for (int col = threadIdx.x; col < c; col += blockDim.x) {
        for (int j0 = 0; j0 <= col; j0 += SL_ROWS) {
            double v[SL_ROWS];
#pragma unroll
            for (int u = 0; u < SL_ROWS; ++u) v[u] = M[(int64_t)min(j0 + u, col) * c + col];
#pragma unroll
            for (int u = 0; u < SL_ROWS; ++u)
                if (j0 + u <= col) slot[tri_index(j0 + u, col, c)] = (SlotT)v[u];
        }
    }
    __syncthreads();
}

template <typename SlotT>
__device__ void slot_store(const SlotT* slot, double* M, int c) {
    for (int col = threadIdx.x; col < c; col += blockDim.x) {
        for (int j0 = 0; j0 < c; j0 += SL_ROWS) {
            double v[SL_ROWS];
#pragma unroll
            for (int u = 0; u < SL_ROWS; ++u) {
                const int j = j0 + u;
                v[u] = j <= col ? (double)slot[tri_index(j, col, c)] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < SL_ROWS; ++u)
                if (j0 + u < c) M[(int64_t)(j0 + u) * c + col] = v[u];
        }
    }
    __syncthreads();
}

// Apply the stored panels np-1 .. p0 (backward) to (slot, A).  Each panel's V and T
// are staged through LDS (two buffers); the global loads run two panels ahead of the
// panel being applied, in two register sets of PF doubles per thread.  When PF values
// per thread cannot hold a panel (few columns, so few threads), a panel is copied
// straight to LDS instead.
template <int BT, typename SlotT, int PF>
__device__ void unfold_tile(SlotT* slot, v4d (&A)[Layout<BT>::RT], int c, int p0, double* lds, const double* store,
                            uint64_t perm) {
    constexpr int VLD = Layout<BT>::VLD, VP = Layout<BT>::VP, TSZ = Layout<BT>::TSZ, PS = Layout<BT>::PS;
    const int wave = qf_group(perm);   // the column tile this wave owns
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
// Leaf fold with a quad of lanes per column (16 rows per lane, quad DPP
// reductions).  The leaves' critical path is the chain of c reflectors per tile:
// the wave that owns a group of 16 columns builds their reflectors one after the
// other, and the other waves apply each one as it is published (q_fold).  The
// reflectors and each panel's T are written in the panel layout of the blocked
// backward pass.
// ---------------------------------------------------------------------------
constexpr int QT = 64;                 // tile rows (matches the blocked pass's BT = 64)
constexpr int LPC = 4;                 // lanes per column
constexpr int RPL = QT / LPC;          // rows per lane: row t = i * LPC + g

// An LDS read issued where it is written: the compiler otherwise moves such reads
// down to their first use, which puts their latency on the reflector chain.
template <typename T>
__device__ __forceinline__ double lds_early(const T* p) {
    typedef __attribute__((address_space(3))) const volatile T lds_t;
    return (double)*(lds_t*)p;
}

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

// Reflector j from (slot[j][j], tile column j held by this quad).  The column goes to
// vbuf unscaled, first, so that its LDS writes overlap the norm and the scalars; the
// scale sc (v = sc x) and tau follow in ts[0..1], tau also in taus_lds[j].  Returns
// sc: a[] keeps x, and the fold scales it to v once the tile is done (the column
// takes no further reflector).
template <typename SlotT, typename RingT>
__device__ __forceinline__ double q_make_reflector(SlotT* slot, const double (&a)[RPL], int c, int j, int g,
                                                   RingT* vbuf, double* ts, double* taus_lds, double& tau_out) {
    const int dj = tri_index(j, j, c);
    const double rjj = lds_early(slot + dj);
#pragma unroll
    for (int i = 0; i < RPL; ++i) vbuf[i * LPC + g] = (RingT)a[i];
    double p4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < RPL; ++i) p4[i & 3] = fma(a[i], a[i], p4[i & 3]);
    const double xn2 = quad_sum((p4[0] + p4[1]) + (p4[2] + p4[3]));
    double tau = 0.0, sc = 0.0;
    if (xn2 > 0.0) {
        // beta = -sign(rjj) |(rjj, x)|, tau = (beta - rjj) / beta = (|rjj| + |beta|) / |beta|,
        // v = x / (rjj - beta).  1 / |beta| is the reciprocal square root already formed;
        // |rjj - beta| = |rjj| + |beta| >= sqrt(xn2) >= 2^-537, so its reciprocal is of a
        // normal number
        const double t = fma(rjj, rjj, xn2);
        const double y = rsqrt_nr(t);
        const double beta = -copysign(t * y, rjj);
        const double u = rjj - beta;
        tau = fabs(u) * y;
        sc = rcp_nr(u);
        if (g == 0) slot[dj] = (SlotT)beta;
    }
    if (g == 0) {
        ts[0] = tau;
        ts[1] = sc;
        taus_lds[j] = tau;
    }
    tau_out = tau;
    return sc;
}

// Reflector j (v = sc x, x the unscaled tile part in LDS) applied to column col:
// w = tau (r + v^T a), r -= w, a -= w v; tsc = tau sc, formed while the dot product
// runs.
template <typename SlotT, typename RingT>
__device__ __forceinline__ void q_reflect_column(SlotT* slot, double (&a)[RPL], int c, int j, int col, int g,
                                                 const RingT* x, double tau, double sc, double tsc) {
    const int idx = tri_index(j, col, c);
    const double r = lds_early(slot + idx);
    double p4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < RPL; ++i) p4[i & 3] = fma(x[i * LPC + g], a[i], p4[i & 3]);
    const double rs = fma(sc, quad_sum((p4[0] + p4[1]) + (p4[2] + p4[3])), r);
    const double w = rs * tau;
    if (g == 0) slot[idx] = (SlotT)(r - w);
    const double ws = rs * tsc;
#pragma unroll
    for (int i = 0; i < RPL; ++i) a[i] = fma(-ws, x[i * LPC + g], a[i]);
}

// LDS of the quad fold: taus_lds[256] | counters ready[QF_RMAX], done[QF_RMAX], abort |
// (tau, sc)[QF_RMAX][PW] | ring[R] of (x[PW][QT_LD], T packed) | slot.  A ring entry
// holds one group's unscaled reflectors (tile parts, row pitch QT_LD), for the waves
// that apply the group one reflector at a time, and the staging of the group's G and
// then T (upper triangle, row-major).  The ring takes what LDS leaves beside the slot,
// 2 to QF_RMAX entries, in sets of two: tile t of a fold uses set t mod m (m = ring / 2),
// its group k the entry k mod 2 of the set (qf_set), so m tiles' chains are in
// flight at once, each alternating between its two entries.  The reflectors
// stay in float64 (RingT): the returned Q has orthonormal columns only as far as the
// fold's R agrees with the stored reflectors, and for a rank-deficient E that
// disagreement is divided by R's tiny diagonal entries, so reflectors rounded to
// float32 where they are applied cost orthonormality (3e-2 measured on a sketch with
// half its columns at noise level).
constexpr int QF_RMAX = 12;
constexpr int QT_LD = QT + 1;
constexpr int QF_TAUS = 0;
constexpr int QF_CNT = QF_TAUS + 256;
constexpr int QF_TS = QF_CNT + QF_RMAX + 1;         // 2 QF_RMAX + 1 unsigned counters (+ pad)
constexpr int QF_X = QF_TS + 2 * PW * QF_RMAX;
constexpr int QF_TPK = PW * (PW + 1) / 2;           // T packed: upper triangle, row-major
// doubles per ring entry: the reflectors in the ring's type, then the T staging
template <typename RingT>
constexpr int qf_xdoubles() { return (PW * QT_LD * (int)sizeof(RingT) + 7) / 8; }
template <typename RingT>
constexpr int qf_entry() { return qf_xdoubles<RingT>() + QF_TPK; }
// Waves k + 1 .. k + QF_SEQ apply group k one reflector at a time, as it is
// published: they build the next groups, so they are on the chain of the fold.  The
// waves further right apply it as one block once its T is published.
constexpr int QF_SEQ = 2;

__device__ __forceinline__ int tpk_index(int i, int j) { return i * PW - (i * (i - 1)) / 2 + (j - i); }
constexpr size_t QF_LDS_LIMIT = 160 * 1024;

template <typename SlotT, typename RingT>
size_t qf_lds_bytes(int c, int ring) {
    return (size_t)(QF_X + ring * qf_entry<RingT>()) * sizeof(double) + (size_t)c * (c + 1) / 2 * sizeof(SlotT);
}

// Groups to waves: group k applies about k - 2 earlier groups as blocks, so the groups
// go, heaviest first, to the SIMD (waves w with w mod 4 = s) with the least work so
// far that still has a wave free.  Packed 4 bits per wave.
uint64_t qf_perm(int np) {
    int load[4] = {0, 0, 0, 0}, used[4] = {0, 0, 0, 0};
    uint64_t perm = 0;
    for (int g = np - 1; g >= 0; --g) {
        int best = -1;
        for (int s = 0; s < 4; ++s) {
            const int w = s + 4 * used[s];
            if (w >= np) continue;
            if (best < 0 || load[s] < load[best]) best = s;
        }
        const int w = best + 4 * used[best];
        perm |= (uint64_t)g << (4 * w);
        load[best] += 3 + std::max(0, g - 2);
        ++used[best];
    }
    return perm;
}

// The deepest ring of whole sets that fits beside the slot, up to three sets (three
// tiles in flight, and fewer when a tile has few groups: LDS left free lets small
// problems share a CU); 0 if not even one set fits.
template <typename SlotT, typename RingT>
int qf_ring(int c) {
    const int want = std::min(QF_RMAX, std::max(2, 2 * std::min(3, ((c + PW - 1) / PW + 1) / 2)));
    for (int r = want; r >= 2; r -= 2)
        if (qf_lds_bytes<SlotT, RingT>(c, r) <= QF_LDS_LIMIT) return r;
    return 0;
}

// Counters in LDS shared by the waves of a workgroup (wrapping, compared by
// difference).  The release operations order a wave's LDS accesses before the
// count, the acquire loads order the count before the waiter's accesses.
typedef __attribute__((address_space(3))) unsigned lds_u32;

__device__ __forceinline__ void q_publish(unsigned* cnt, unsigned value) {
    __hip_atomic_store((lds_u32*)cnt, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A count published without a hardware wait: the LDS executes a wave's operations in
// the order they are issued, so a waiter that sees the count (by an acquire load) also
// sees every LDS write the publishing wave issued before it.  Only the compiler must
// be kept from moving those writes past the count.
__device__ __forceinline__ void q_publish_inorder(unsigned* cnt, unsigned value) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store((lds_u32*)cnt, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void q_arrive(unsigned* cnt) {
    __hip_atomic_fetch_add((lds_u32*)cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Every wait is bounded: after QF_SPIN_CAP polls (far beyond any legitimate wait:
// the longest is one wave waiting for another's share of a tile) the wave raises the
// workgroup's abort flag, and every wait returns at once once the flag is up, so a
// broken protocol ends the kernel with BFGS_ERR_NUMERIC instead of hanging.
constexpr unsigned QF_SPIN_CAP = 1u << 22;

__device__ __forceinline__ bool q_aborted(const unsigned* abort_flag) {
    return __hip_atomic_load((lds_u32*)abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u;
}

__device__ __forceinline__ void q_wait(unsigned* cnt, unsigned value, unsigned* abort_flag) {
    unsigned polls = 0;
    while ((int)(__hip_atomic_load((lds_u32*)cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) - value) < 0) {
        if (q_aborted(abort_flag)) return;
        if (++polls == QF_SPIN_CAP) {
            __hip_atomic_store((lds_u32*)abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Wait until the counter, read as a signed value, is no longer negative.
__device__ __forceinline__ void q_wait_nonneg(unsigned* cnt, unsigned* abort_flag) {
    unsigned polls = 0;
    while ((int)__hip_atomic_load((lds_u32*)cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < 0) {
        if (q_aborted(abort_flag)) return;
        if (++polls == QF_SPIN_CAP) {
            __hip_atomic_store((lds_u32*)abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// q_wait for a counter whose last value seen by this wave is `seen`: no load when
// that already covers `value` (an acquire that saw a count orders everything
// released up to it); otherwise wait and keep the new value.
__device__ __forceinline__ void q_wait_seen(unsigned* cnt, unsigned value, unsigned& seen, unsigned* abort_flag) {
    unsigned polls = 0;
    while ((int)(seen - value) < 0) {
        seen = __hip_atomic_load((lds_u32*)cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if ((int)(seen - value) < 0) {
            if (q_aborted(abort_flag)) return;
            if (++polls == QF_SPIN_CAP) {
                __hip_atomic_store((lds_u32*)abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

// Ring entries come in m = ring / 2 sets of two: tile t of a fold takes set t mod m
// and its group k the entry k mod 2 of the set, so m tiles' chains are in flight at
// once, each alternating between its two entries.  Group (t, k) counts
// 256 (t np + k) + 1 + (reflectors published) in its entry's ready counter, so the
// counts of an entry only grow from one group to the next.  The entry's previous
// group is (t, k - 2) if the tile has it, else the last group of tile t - m with the
// parity of k (a fold's tiles start at group k0 = 0 for the leaves and 4 t for a tree
// combine, never later than the tile before, so tile t - m has that group), else
// none.  qf_prev_first returns that group's first count, or 0 for none (a first count
// is never 0).
__device__ __forceinline__ int qf_set(int t, int ring) { return (t % (ring >= 2 ? ring / 2 : 1)) * 2; }

__device__ __forceinline__ unsigned qf_prev_first(unsigned tag, int k, int k0, int np, int ring) {
    if (k - 2 >= k0) return tag - 512u;
    // the tags of m tiles: group (t, k) has a tile t - m iff its tag exceeds them
    const unsigned back = (unsigned)((ring >= 2 ? ring / 2 : 1) * np) * 256u;
    if (tag <= back) return 0u;
    return tag - back + (unsigned)((np - 1 - k) >> 1) * 512u;
}

// A wave's tile columns in two layouts.  Quad layout (reflector building and the
// one-at-a-time application): lane 4 j + g holds rows 4 i + g of the wave's column j
// in a[i].  Matrix-core layout (block application): lane 16 q + j holds rows 4 i + q
// of column j in a[i], which is at once the B operand of v_mfma_f64_16x16x4f64 for
// k-step i and, read as four 16-row output tiles, its accumulator layout.  Going
// from one to the other is a lane permutation with the register index unchanged.
__device__ __forceinline__ void quad_to_mfma(double (&a)[RPL]) {
    const int lane = fresh_lane();
    const int src = 4 * (lane & 15) + (lane >> 4);
#pragma unroll
    for (int i = 0; i < RPL; ++i) a[i] = bpermute_f64(a[i], src);
}

__device__ __forceinline__ void mfma_to_quad(double (&a)[RPL]) {
    const int lane = fresh_lane();
    const int src = 16 * (lane & 3) + (lane >> 2);
#pragma unroll
    for (int i = 0; i < RPL; ++i) a[i] = bpermute_f64(a[i], src);
}

// The compact-WY factor of this wave's panel (its 16 columns = one group, scaled
// v = sc x, in quad layout), written to Tb (upper triangle, packed) and returned in
// trow (lane r < 16: row r).  G = V^T V is formed on the matrix cores (V's rows
// 4 ks .. 4 ks + 3 sit in a[ks] of the quads, one lane permutation away from the
// operand layout) and its upper triangle stored to Tb; every lane then reads the G
// entries it needs from there (the same address in every lane), lane r forms row r
// of T (I - V T V^T, upper triangular) and T replaces G in Tb.  A wave's LDS
// operations complete in order, so the reads of G precede the writes of T.
__device__ __forceinline__ void q_panel_t(const double (&a)[RPL], int c, const double* taus_lds, double* Tb,
                                          double (&trow)[PW], uint64_t perm) {
    const int wave = qf_group(perm), lane = fresh_lane();
    const int src = 4 * (lane & 15) + (lane >> 4);
    v4d gacc = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < RPL; ++ks) {
        const double v = bpermute_f64(a[ks], src);
        gacc = mfma64(v, v, gacc);
    }
    // lane 16 m + i holds G(4 reg + m, i) in gacc[reg]
    const int gi = lane & 15, gm = lane >> 4;
#pragma unroll
    for (int reg = 0; reg < 4; ++reg)
        if (4 * reg + gm <= gi) Tb[tpk_index(4 * reg + gm, gi)] = gacc[reg];
    const int r = lane & 15;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int ci = wave * PW + i;             // < 256: taus_lds[ci] exists
        const double tau_r = lds_early(taus_lds + ci);
        const double tau_i = ci < c ? tau_r : 0.0;
        double sacc = 0.0;
        // volatile reads, in order: merged and hoisted, the 120 reads of G would take
        // 240 registers
#pragma unroll
        for (int b = 0; b < i; ++b) sacc = fma(trow[b], lds_early(Tb + tpk_index(b, i)), sacc);
        // rows above r come out zero: every term of their sums is
        trow[i] = i == r ? tau_i : -tau_i * sacc;
    }
    if (lane < PW) {
#pragma unroll
        for (int i = 0; i < PW; ++i)
            if (i >= lane) Tb[tpk_index(lane, i)] = trow[i];
    }
}

// Group (reflectors jb .. jb + 15) applied at once to this wave's columns, held in
// the matrix-core layout, and to their slot rows jb .. jb + 15, read from the group's
// stored panel: V (16 columns of 64 tile rows, v = sc x, column-major) and the full
// 16 x 16 T (row-major), both zero past the group's ng reflectors.  With the slot
// part of reflector i the unit row, the group's product is I - V T V^T, and applying
// H_jb first, then H_jb+1, ... is its transpose:
//   W = S_p + V^T A;  W' = T^T W;  S_p -= W';  A -= V W'.
// Every product is a v_mfma_f64_16x16x4f64 chain: 16 + 4 + 16 per group.
template <typename SlotT>
__device__ __forceinline__ void q_block_apply(SlotT* slot, double (&a)[RPL], int c, int jb, int ng,
                                              const double* __restrict__ panel, uint64_t perm) {
    const int lane = fresh_lane(), jl = lane & 15, q = lane >> 4, wave = qf_group(perm);
    const int colw = wave * PW + jl;
    const bool colok = colw < c;
    const double* V = panel;
    const double* T = panel + PW * QT;
    double xa[RPL];
#pragma unroll
    for (int ks = 0; ks < RPL; ++ks) xa[ks] = V[jl * QT + 4 * ks + q];   // V(4 ks + q, jl)
    v4d wt = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < RPL; ++ks) wt = mfma64(xa[ks], a[ks], wt);
    double tv[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) tv[ks] = T[(4 * ks + q) * PW + jl];   // T(4 ks + q, jl)
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int m = 0; m < 4; ++m) xa[4 * blk + m] = V[(4 * m + q) * QT + 16 * blk + jl];   // V(16 blk + jl, 4 m + q)
    v4d w;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = q + 4 * r;
        const double sp = (colok && i < ng) ? (double)slot[tri_index(jb + i, colw, c)] : 0.0;
        w[r] = wt[r] + sp;
    }
    v4d wp = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) wp = mfma64(tv[ks], w[ks], wp);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = q + 4 * r;
        if (colok && i < ng) {
            const int idx = tri_index(jb + i, colw, c);
            slot[idx] = (SlotT)((double)slot[idx] - wp[r]);
        }
    }
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
        v4d acc = {a[4 * blk], a[4 * blk + 1], a[4 * blk + 2], a[4 * blk + 3]};
#pragma unroll
        for (int m = 0; m < 4; ++m) acc = mfma64(-xa[4 * blk + m], wp[m], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) a[4 * blk + r] = acc[r];
    }
}

// Fold the tile held in a[] (this quad's column, quad layout) into the slot with
// reflectors j0 .. c-1 (the tile's columns below j0 are zero; j0 is a multiple of PW).
// Reflectors come in groups of PW: group k (reflectors PW k .. PW k + PW - 1) is
// built by wave k, which owns those columns, one reflector after the other, each
// applied to the wave's later columns at once (a wave's LDS operations complete in
// order, so its own writes need no synchronisation).  Group k of the fold's tile t
// takes entry k mod 2 of the ring's set t mod (ring / 2).  Each reflector is
// published in its entry's ready counter (value 256 (t np + k) + slot + 1) as soon as
// it is written; once the group is complete its builder forms the group's compact-WY
// factor T, stores the panel (V, T) to `panels` and, once those stores are complete,
// publishes one count more.  Waves k + 1 .. k + QF_SEQ, the next groups' builders,
// apply each reflector as it is published (they are on the chain of the fold); the
// waves further right wait for the final count and apply the whole group as one
// block on the matrix cores (q_block_apply), holding their columns in the
// matrix-core layout until they reach the first group they apply one at a time.
// Every wave that used a group (its builder included) arrives at the entry's done
// counter afterwards; the wave that next fills the entry first waits for all of
// them, so one builder at a time writes an entry and its ready counter only grows.
// A wave is done with a tile once it has built its own group, and goes on to the
// next tile: the chains of ring / 2 tiles overlap, each in its own set of entries.
// No wave shares slot entries with another (an entry belongs to its
// column's wave), so there is no barrier: each wait is for an event of an earlier
// group, whose waves wait only for still earlier ones, so every wait ends.
template <typename SlotT, typename RingT>
__device__ __forceinline__ void q_fold(SlotT* slot, double (&a)[RPL], int c, int j0, double* xring,
                                       double* tsring, double* taus_lds, unsigned* cnt, int ring, int t,
                                       double* panels, uint64_t perm) {
    const int wave = qf_group(perm);   // = col / PW
    const int np = (c + PW - 1) / PW;
    const int k0 = j0 / PW;
    unsigned* abort_flag = cnt + 2 * QF_RMAX;
    double sc_own = 0.0;                 // the scale of this quad's reflector (columns j0 .. c-1)
    const bool block_first = wave >= k0 + QF_SEQ + 1;
    if (block_first) quad_to_mfma(a);
    const int set = qf_set(t, ring);
    unsigned tag = (unsigned)(t * np + k0) * 256u + 1u;   // group k's first count
    for (int k = k0; k < np; ++k, tag += 256u) {
        const int lane_k = fresh_lane();
        const int col = wave * PW + (lane_k >> 2), g = lane_k & 3;   // as the caller's, re-formed
        const int jb = k * PW, je = min(jb + PW, c), ng = je - jb;
        const int r = set + (k & 1);
        RingT* xb = (RingT*)(xring + r * qf_entry<RingT>());
        double* Tb = xring + r * qf_entry<RingT>() + qf_xdoubles<RingT>();
        double* tb = tsring + r * 2 * PW;
        unsigned* ready = cnt + r;
        unsigned* done = cnt + QF_RMAX + r;
        if (wave >= k) {
            if (wave == k) {
                const unsigned prev = qf_prev_first(tag, k, k0, np, ring);
                if (prev != 0u) {
                    // the entry's previous group: once its builder has published (and so
                    // has set done to minus its users), done back at zero means every
                    // user has arrived
                    q_wait(ready, prev, abort_flag);
                    q_wait_nonneg(done, abort_flag);
                }
                // this group's slot users: the builder and the waves that apply it one
                // reflector at a time (ordered before the first publication by its
                // release)
                if ((threadIdx.x & 63) == 0)
                    __hip_atomic_store((lds_u32*)done, (unsigned)(-(1 + min(QF_SEQ, np - 1 - k))), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                // the builder carries the chain of reflectors: it goes first on its SIMD
                __builtin_amdgcn_s_setprio(2);
                for (int j = jb; j < je; ++j) {
                    const int sl = j - jb;   // quad sl of this wave holds column j
                    double tau_q = 0.0, sc_q = 0.0;
                    if (col == j) {
                        sc_q = q_make_reflector(slot, a, c, j, g, xb + sl * QT_LD, tb + 2 * sl, taus_lds, tau_q);
                        sc_own = sc_q;
                    }
                    // publish the reflector for the waves that apply the group one
                    // reflector at a time (no wait, see q_publish_inorder)
                    if (fresh_lane() == 0) q_publish_inorder(ready, tag + (unsigned)sl);
                    // the scalars straight from quad sl's registers, x from the ring (the
                    // 16 quads read the same 4 addresses per instruction, a broadcast)
                    const double tau = read_lane(tau_q, 4 * sl), sc = read_lane(sc_q, 4 * sl);
                    // tau = 0 (a zero column) leaves the column and the slot as they are
                    if (col > j && col < c) q_reflect_column(slot, a, c, j, col, g, xb + sl * QT_LD, tau, sc, tau * sc);
                }
                __builtin_amdgcn_s_setprio(0);
                // x -> v (zero stays zero for a zero column, sc = 0); the group's T beside
                // its reflectors, then the count the block consumers wait for
#pragma unroll
                for (int i = 0; i < RPL; ++i) a[i] *= sc_own;
                double trow[PW];
                q_panel_t(a, c, taus_lds, Tb, trow, perm);
                const int lane = fresh_lane();
                // the panel (V, T) for the block appliers and the backward pass; the
                // count that releases the block appliers follows once it is written
                double* dst = panels + (int64_t)k * Layout<QT>::PS;
#pragma unroll
                for (int i = 0; i < RPL; ++i) dst[(col % PW) * QT + i * LPC + g] = a[i];
                if (lane < PW) {
#pragma unroll
                    for (int i = 0; i < PW; ++i) dst[PW * QT + lane * PW + i] = trow[i];
                }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                if (lane == 0) q_publish(ready, tag + (unsigned)ng);
            } else if (wave <= k + QF_SEQ) {
                // the next groups' builders apply this group as it is published
                if (block_first && wave == k + QF_SEQ) mfma_to_quad(a);
                unsigned seen = tag - 1u;   // nothing of this group seen yet
                if (wave == k + 1) __builtin_amdgcn_s_setprio(1);
                for (int j = jb; j < je; ++j) {
                    const int sl = j - jb;
                    q_wait_seen(ready, tag + (unsigned)sl, seen, abort_flag);
                    const double tau = lds_early(tb + 2 * sl), sc = lds_early(tb + 2 * sl + 1);
                    if (col < c) q_reflect_column(slot, a, c, j, col, g, xb + sl * QT_LD, tau, sc, tau * sc);
                }
                __builtin_amdgcn_s_setprio(0);
            } else {
                // counts only grow: a later group's count in this slot also means
                // this group's panel is stored
                q_wait(ready, tag + (unsigned)ng, abort_flag);
                q_block_apply(slot, a, c, jb, ng, panels + (int64_t)k * Layout<QT>::PS, perm);
            }
            if (wave <= k + QF_SEQ && threadIdx.x % 64 == 0) q_arrive(done);
        }
    }
}

template <typename TE, typename SlotT>
__global__ void __launch_bounds__(1024) leaf_forward_q(int64_t n, int c, int64_t rows_per_chain,
                                                       const TE* __restrict__ E, double* __restrict__ refl,
                                                       double* __restrict__ Rs, int ring, int32_t* __restrict__ status,
                                                       uint64_t perm) {
    extern __shared__ double lds[];
    double* xring = lds + QF_X;
    double* tsring = lds + QF_TS;
    double* taus_lds = lds + QF_TAUS;
    unsigned* cnt = (unsigned*)(lds + QF_CNT);
    SlotT* slot = (SlotT*)(lds + QF_X + ring * qf_entry<double>());
    if (threadIdx.x <= 2 * QF_RMAX) cnt[threadIdx.x] = 0;   // counters and the abort flag; the slot set-up's barrier follows
    constexpr int PS = Layout<QT>::PS;
    const int ch = blockIdx.x, col = qf_group(perm) * PW + (threadIdx.x & 63) / LPC, g = threadIdx.x % LPC;
    const int np = (c + PW - 1) / PW;
    const int64_t r_begin = ch * rows_per_chain;
    const int64_t r_end = min(n, r_begin + rows_per_chain);
    const int tiles_per_chain = (int)(rows_per_chain / QT);
    slot_zero(slot, c);
    // Every load of E is issued (clamped to an element of E) and masked after it: a
    // conditional load would be waited for on its own.  The tile is loaded when the
    // wave starts it (the other waves' work covers the latency; a prefetch of the
    // next tile would hold 16 more registers through the fold, which has none left).
    const int colc = min(col, c - 1);
    for (int tile = 0; r_begin + (int64_t)tile * QT < r_end; ++tile) {
        const int64_t r0 = r_begin + (int64_t)tile * QT;
        TE nx[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) nx[i] = E[(int64_t)colc * n + min(r0 + i * LPC + g, r_end - 1)];
        double a[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int64_t r = r0 + i * LPC + g;
            a[i] = (col < c && r < r_end) ? to_f64(nx[i]) : 0.0;
        }
        const int64_t gtile = (int64_t)ch * tiles_per_chain + tile;
        q_fold<SlotT, double>(slot, a, c, 0, xring, tsring, taus_lds, cnt, ring, tile, refl + gtile * np * PS, perm);
        if (q_aborted(cnt + 2 * QF_RMAX)) break;
    }
    __syncthreads();   // the folds have no barrier; slot_store reads every column's entries
    if (threadIdx.x == 0 && q_aborted(cnt + 2 * QF_RMAX)) set_status(status, BFGS_ERR_NUMERIC);
    slot_store(slot, Rs + (int64_t)ch * c * c, c);
}

// Tree fold with the quad scheme: combine i of a level folds R_b (chain a + stride)
// into the slot holding R_a, 64 rows at a time; tile t of R_b is zero left of
// column 64 t, so its reflectors start there.  Its panels p >= 64 t / 16 go to
// tree + ((comb_off + i) * ntt + t) * np * PS + p * PS, as the backward pass reads them.
template <typename SlotT>
__global__ void __launch_bounds__(1024) tree_forward_q(int c, int stride, int64_t comb_off, double* __restrict__ Rs,
                                                       double* __restrict__ tree, int ring, int32_t* __restrict__ status,
                                                       uint64_t perm) {
    extern __shared__ double lds[];
    double* xring = lds + QF_X;
    double* tsring = lds + QF_TS;
    double* taus_lds = lds + QF_TAUS;
    unsigned* cnt = (unsigned*)(lds + QF_CNT);
    SlotT* slot = (SlotT*)(lds + QF_X + ring * qf_entry<double>());
    if (threadIdx.x <= 2 * QF_RMAX) cnt[threadIdx.x] = 0;   // counters and the abort flag; the slot set-up's barrier follows
    constexpr int PS = Layout<QT>::PS;
    const int i = blockIdx.x, col = qf_group(perm) * PW + (threadIdx.x & 63) / LPC, g = threadIdx.x % LPC;
    const int np = (c + PW - 1) / PW, ntt = (c + QT - 1) / QT;
    const int a_idx = i * 2 * stride, b_idx = a_idx + stride;
    const double* Rb = Rs + (int64_t)b_idx * c * c;
    slot_load(slot, Rs + (int64_t)a_idx * c * c, c);
    for (int t = 0; t < ntt; ++t) {
        double a[RPL];
        const int colc = min(col, c - 1);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int row = t * QT + q * LPC + g;
            const double v = Rb[(int64_t)min(row, c - 1) * c + colc];   // clamped, masked below
            a[q] = (col < c && row < c && col >= row) ? v : 0.0;
        }
        q_fold<SlotT, double>(slot, a, c, t * QT, xring, tsring, taus_lds, cnt, ring, t,
               tree + ((comb_off + i) * ntt + t) * np * PS, perm);
        if (q_aborted(cnt + 2 * QF_RMAX)) break;
    }
    __syncthreads();   // the folds have no barrier; slot_store reads every column's entries
    if (threadIdx.x == 0 && q_aborted(cnt + 2 * QF_RMAX)) set_status(status, BFGS_ERR_NUMERIC);
    slot_store(slot, Rs + (int64_t)a_idx * c * c, c);
}

// ---------------------------------------------------------------------------
// Kernels of the blocked passes.  Leaf tile g of chain ch stores its panels at
// refl + (g * np + p) * PS.
// ---------------------------------------------------------------------------
template <typename TQ, typename SlotT, int BT, int PF>
__global__ void __launch_bounds__(1024) leaf_backward(int64_t n, int c, int64_t rows_per_chain,
                                                      const double* __restrict__ refl, const double* __restrict__ Qtop,
                                                      TQ* __restrict__ Q, uint64_t perm, int qblk) {
    extern __shared__ double lds[];
    constexpr int RT = Layout<BT>::RT, PS = Layout<BT>::PS;
    SlotT* slot = (SlotT*)(lds + Layout<BT>::HEAD);
    const int ch = blockIdx.x, lane = threadIdx.x & 63, jl = lane & 15, q = lane >> 4;
    const int np = (c + PW - 1) / PW;
    const int col = qf_group(perm) * PW + jl;
    const int64_t r_begin = ch * rows_per_chain;
    if (r_begin >= n) return;   // uniform: whole workgroup leaves
    const int64_t r_end = min(n, r_begin + rows_per_chain);
    const int tiles_per_chain = (int)(rows_per_chain / BT);
    const int ntiles = (int)((r_end - r_begin + BT - 1) / BT);
    // column-major Q (leading dimension n), or the chain's own block of Q (leading
    // dimension rows_per_chain)
    TQ* Qc = qblk ? Q + (int64_t)ch * rows_per_chain * c - r_begin : Q;
    const int64_t ldq = qblk ? rows_per_chain : n;
    slot_load(slot, Qtop + (int64_t)ch * c * c, c);
    for (int tile = ntiles - 1; tile >= 0; --tile) {
        const int64_t r0 = r_begin + (int64_t)tile * BT;
        const int64_t gtile = (int64_t)ch * tiles_per_chain + tile;
        v4d A[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) A[rt] = v4d{0, 0, 0, 0};
        unfold_tile<BT, SlotT, PF>(slot, A, c, 0, lds, refl + gtile * np * PS, perm);
        if (col < c) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = r0 + rt * 16 + q + 4 * r;
                    if (row < r_end) Qc[(int64_t)col * ldq + row] = (TQ)A[rt][r];
                }
        }
    }
}

// Tree backward: combine i of a level (chain a = i * 2 * stride, b = a + stride)
// applies the panels tree_forward_q stored for its tiles t (rows t * BT .. of R_b).
template <typename SlotT, int BT, int PF>
__global__ void __launch_bounds__(1024) tree_backward(int c, int stride, int64_t comb_off, double* __restrict__ Qtop,
                                                      const double* __restrict__ tree, uint64_t perm) {
    extern __shared__ double lds[];
    constexpr int RT = Layout<BT>::RT, PS = Layout<BT>::PS;
    SlotT* slot = (SlotT*)(lds + Layout<BT>::HEAD);
    const int i = blockIdx.x, lane = threadIdx.x & 63, jl = lane & 15, q = lane >> 4;
    const int np = (c + PW - 1) / PW, ntt = (c + BT - 1) / BT;
    const int col = qf_group(perm) * PW + jl;
    const int a_idx = i * 2 * stride, b_idx = a_idx + stride;
    double* Qb = Qtop + (int64_t)b_idx * c * c;
    slot_load(slot, Qtop + (int64_t)a_idx * c * c, c);
    for (int t = ntt - 1; t >= 0; --t) {
        v4d A[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) A[rt] = v4d{0, 0, 0, 0};
        unfold_tile<BT, SlotT, PF>(slot, A, c, (t * BT) / PW, lds, tree + ((comb_off + i) * ntt + t) * np * PS, perm);
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
template <typename TE, typename TQ, typename SlotT, int BT, int PF>
int tsqr_impl(bfgsuq_ctx* h, int c, const TE* E, TQ* Q, double** R_out, bool q_blocked) {
    static_assert(BT == QR_TILE, "chain rows are counted in QR_TILE-row tiles");
    constexpr int PS = Layout<BT>::PS;
    const int64_t n = h->n;
    const int np = (c + PW - 1) / PW;
    const int threads = 64 * np;
    int nchains;
    const int64_t rows_per_chain = tsqr_chain_rows(h, &nchains);
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
        if (hipFuncSetAttribute((const void*)leaf_backward<TQ, SlotT, BT, PF>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
            hipFuncSetAttribute((const void*)tree_forward_q<SlotT>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess ||
            hipFuncSetAttribute((const void*)tree_backward<SlotT, BT, PF>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
            return BFGS_ERR_HIP;
        attr_done = true;
    }
    static bool attr_q = false;
    if (!attr_q) {
        if (hipFuncSetAttribute((const void*)leaf_forward_q<TE, SlotT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024) != hipSuccess)
            return BFGS_ERR_HIP;
        attr_q = true;
    }
    // float64 rings in both folds (>= 2 entries: the slot type was chosen for that)
    const int ring = qf_ring<SlotT, double>(c);
    const int tring = ring;
    const uint64_t perm = qf_perm(np);
    if (ring < 2) return BFGS_ERR_ARG;
    const size_t leaf_lds = qf_lds_bytes<SlotT, double>(c, ring), tree_lds = leaf_lds;
    prof_begin(h, "tsqr_leaf_fwd");
    hipLaunchKernelGGL((leaf_forward_q<TE, SlotT>), dim3(nchains), dim3(LPC * 16 * np), leaf_lds,
                       h->stream, n, c, rows_per_chain, E, refl, Rs, ring, h->status, perm);
    prof_end(h);
    prof_begin(h, "tsqr_tree");
    int64_t off = 0;
    for (int stride = 1; stride < nchains; stride *= 2) {
        const int ncomb = nchains / (2 * stride);
        hipLaunchKernelGGL((tree_forward_q<SlotT>), dim3(ncomb), dim3(threads), tree_lds,
                           h->stream, c, stride, off, Rs, tree, tring, h->status, perm);
        off += ncomb;
    }
    hipLaunchKernelGGL(set_identity_kernel, dim3(64), dim3(256), 0, h->stream, Qtop, c);
    for (int stride = nchains / 2; stride >= 1; stride /= 2) {
        const int ncomb = nchains / (2 * stride);
        off -= ncomb;
        hipLaunchKernelGGL((tree_backward<SlotT, BT, PF>), dim3(ncomb), dim3(threads), smem, h->stream, c, stride, off,
                           Qtop, tree, perm);
    }
    prof_end(h);
    prof_begin(h, "tsqr_leaf_bwd");
    hipLaunchKernelGGL((leaf_backward<TQ, SlotT, BT, PF>), dim3(nchains), dim3(threads), smem, h->stream, n, c,
                       rows_per_chain, refl, Qtop, Q, perm, q_blocked ? 1 : 0);
    prof_end(h);
    *R_out = Rs;   // chain 0 holds the final R (row-major, upper triangular)
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

template <typename TE, typename TQ>
int tsqr_dispatch(bfgsuq_ctx* h, int c, const TE* E, TQ* Q, double** R_out, bool q_blocked) {
    if (c < 1 || c > 256) return BFGS_ERR_ARG;
    // 64-row tiles keep a tile's fragments, the staging registers and the panel work
    // within 128 registers per lane (1024-thread workgroups); the slot is float64
    // whenever it fits in LDS (c <= 184) and float32 above that
    const size_t lim = 160 * 1024;
    const bool dslot = lds_bytes<64, double>(c) <= lim && qf_ring<double, double>(c) >= 2;
    // staging doubles per thread for one stored panel (64 * ceil(c / 16) threads); more
    // than 8 (c <= 32) copies panels straight to LDS
    const int pf = ceil_div(Layout<64>::PS, 64 * ceil_div(c, PW));
    if (pf <= 2) return dslot ? tsqr_impl<TE, TQ, double, 64, 2>(h, c, E, Q, R_out, q_blocked) : tsqr_impl<TE, TQ, float, 64, 2>(h, c, E, Q, R_out, q_blocked);
    if (pf <= 3) return dslot ? tsqr_impl<TE, TQ, double, 64, 3>(h, c, E, Q, R_out, q_blocked) : tsqr_impl<TE, TQ, float, 64, 3>(h, c, E, Q, R_out, q_blocked);
    if (pf <= 5) return dslot ? tsqr_impl<TE, TQ, double, 64, 5>(h, c, E, Q, R_out, q_blocked) : tsqr_impl<TE, TQ, float, 64, 5>(h, c, E, Q, R_out, q_blocked);
    return dslot ? tsqr_impl<TE, TQ, double, 64, 8>(h, c, E, Q, R_out, q_blocked) : tsqr_impl<TE, TQ, float, 64, 8>(h, c, E, Q, R_out, q_blocked);
}

}  // namespace

bool tsqr_f64_slot(int c) {
    return c >= 1 && c <= 256 && lds_bytes<64, double>(c) <= 160 * 1024 && qf_ring<double, double>(c) >= 2;
}

extern "C" int bfgs_tsqr_shape(int32_t c, int32_t* slot_f64, int32_t* ring) {
    if (c < 1 || c > BFGS_MAX_COLS) return BFGS_ERR_ARG;
    const bool dslot = tsqr_f64_slot(c);
    if (slot_f64) *slot_f64 = dslot ? 1 : 0;
    if (ring) *ring = dslot ? qf_ring<double, double>(c) : qf_ring<float, double>(c);
    return BFGS_OK;
}

int64_t tsqr_chain_rows(const bfgsuq_ctx* h, int* nchains) {
    const int64_t tiles_total = (h->n + QR_TILE - 1) / QR_TILE;
    const int nch = (int)std::min<int64_t>(h->qr_chains, floor_pow2(std::max<int64_t>(1, tiles_total / 2)));
    if (nchains) *nchains = nch;
    return round_up((h->n + nch - 1) / nch, QR_TILE);
}

int tsqr_run(bfgsuq_ctx* h, int c, const float* E, float* Q, double** R_out, bool q_blocked) {
    return tsqr_dispatch(h, c, E, Q, R_out, q_blocked);
}
int tsqr_run(bfgsuq_ctx* h, int c, const double* E, float* Q, double** R_out) {
    return tsqr_dispatch(h, c, E, Q, R_out, false);
}
int tsqr_run(bfgsuq_ctx* h, int c, const double* E, double* Q, double** R_out) {
    return tsqr_dispatch(h, c, E, Q, R_out, false);
}
