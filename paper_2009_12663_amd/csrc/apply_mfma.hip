// B_k V for bfloat16 storage on the CDNA4 matrix cores.
//
// Same compact form as apply.hip (two streaming passes over S and Y around a
// float64 k x k solve), with both passes as bfloat16 MFMA (32x32x16, float32
// accumulation) over layouts written at push time so that every wave's operand
// load is one contiguous 1 KB block:
//
//   F1 (pass 1, contraction over rows): 16-row blocks, pair-major inside:
//        element (r, p) at (r / 16) * kmax * 16 + p * 16 + r % 16
//   F2 (pass 2, contraction over pairs): 32-row blocks of 16-pair groups:
//        element (r, p) at (r / 32) * G * 512 + (p / 16) * 512 + (r % 32) * 16 + p % 16
//        with G = ceil(kmax / 16) groups (missing pairs are zero)
//
// Pass 1:  Z_s = S^T V and Z_y = Y^T (B_0 V).  One workgroup per (row range,
//          S or Y); the S and Y workgroups of a row range sit on the same XCD so
//          the V block they both stage through LDS is read from HBM once.  With
//          a diagonal B_0 the Y workgroup multiplies V by h0 in float32 and
//          splits the product into bfloat16 hi + lo (two MFMAs); with B_0 = gamma I
//          the scale is applied in float64 after the reduction.
// Pass 2:  computed transposed, out^T = small^T W^T, so that a lane owns one
//          output row and all writes are coalesced.  The small operand is
//          [-P ; T] split into bfloat16 hi + lo (the float64 solve result would
//          otherwise lose 8 bits); the Y half is accumulated first, the
//          accumulator is scaled by h0[row] (one per lane), then the S half
//          is added: out = h0 o (V - Y P) + S T.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

struct alignas(16) u16x8 {
    uint16_t v[8];
};

__device__ __forceinline__ bf16x8 as_bf16x8(const uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ __forceinline__ floatx16 mfma32(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t bf16_bits_rne(float f) { return float_to_bf16(f).bits; }
__device__ __forceinline__ float bits_to_f32(uint16_t b) {
    bf16_t h;
    h.bits = b;
    return bf16_to_float(h);
}

// ---------------------------------------------------------------------------
// Push: scatter stored column j into F1 and F2.
// ---------------------------------------------------------------------------
__global__ void scatter_pair_layouts(int64_t n, int64_t rows_f1, int64_t rows_f2, int kmax, int G, int j,
                                     const bf16_t* __restrict__ Scol, const bf16_t* __restrict__ Ycol,
                                     bf16_t* __restrict__ S1, bf16_t* __restrict__ Y1, bf16_t* __restrict__ S2,
                                     bf16_t* __restrict__ Y2) {
    const int64_t rows = rows_f1 > rows_f2 ? rows_f1 : rows_f2;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        bf16_t s, y;
        s.bits = 0;
        y.bits = 0;
        if (r < n) {
            s = Scol[r];
            y = Ycol[r];
        }
        if (r < rows_f1) {
            const int64_t o = (r / 16) * (int64_t)kmax * 16 + (int64_t)j * 16 + r % 16;
            S1[o] = s;
            Y1[o] = y;
        }
        if (r < rows_f2) {
            const int64_t o = (r / 32) * (int64_t)G * 512 + (int64_t)(j / 16) * 512 + (r % 32) * 16 + j % 16;
            S2[o] = s;
            Y2[o] = y;
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 1
// ---------------------------------------------------------------------------
// Rows per stage: 128 (8 MFMA k-steps of 16) while the register budget allows it,
// 64 from six column tiles.  Two stages are in flight while a third is used: each
// register set is refilled as soon as its stage is consumed (V once staged in LDS, the
// pair fragments once multiplied).
template <int NT>
struct G1Shape {
    static constexpr int STAGE = NT >= 6 ? 64 : 128;
    static constexpr int KS = STAGE / 16;
    static constexpr int CPC = STAGE / 8;   // 16-byte chunks per staged V column
    static constexpr int LD = STAGE + 8;    // LDS pitch (elements) of a staged V column
};
int g1_stage(int NT) { return NT >= 6 ? G1Shape<8>::STAGE : G1Shape<1>::STAGE; }

// blockDim = 64 * MT (one 32-pair tile per wave); grid = 16 * ceil(nk / 8)
template <int NT, bool DIAG>
__global__ void __launch_bounds__(512) gemm1_mfma(int64_t n, int k, int kmax, int c, const bf16_t* __restrict__ S1,
                                                  const bf16_t* __restrict__ Y1, const float* __restrict__ h0,
                                                  const bf16_t* __restrict__ V, float* __restrict__ part,
                                                  int64_t rows_per_xcd, int64_t rows_f1, int nk, int v_aligned) {
    constexpr int G1_STAGE = G1Shape<NT>::STAGE, G1_KS = G1Shape<NT>::KS, G1_CPC = G1Shape<NT>::CPC;
    constexpr int VS_LD = G1Shape<NT>::LD;
    extern __shared__ unsigned char smem_raw[];
    uint16_t* Vs = (uint16_t*)smem_raw;                 // [NT*32][VS_LD]
    uint16_t* Vl = Vs + NT * 32 * VS_LD;                // low halves (Y part, diagonal B_0)
    // Workgroup g runs on XCD g % 8.  Each XCD owns a contiguous eighth of the rows
    // (rows_per_xcd, a whole number of stages) and deals its stages round-robin to its
    // nk / 8 row slots, so the slots of one XCD stream neighbouring rows of every V
    // column together.  The S and Y workgroups of a slot (g and g + 8) share an XCD,
    // and with it the V stage in L2.
    const int g = blockIdx.x;
    const int xcd = g % 8, slot = g / 8, nj = nk / 8;
    const int part_id = slot % 2, j = slot / 2;
    if (j >= nj) return;                                 // whole workgroup
    const int kr = xcd * nj + j;                         // partial-sum index
    const bool scaled = DIAG && part_id == 1;
    const bf16_t* W = part_id ? Y1 : S1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int p = wave * 32 + (lane & 31);               // pair owned by this lane in the A fragment
    const bool active = wave * 32 < k;                   // waves past the last pair tile only stage V
    const int half = lane >> 5;
    const int64_t r_begin = (int64_t)xcd * rows_per_xcd + (int64_t)j * G1_STAGE;
    int64_t r_end = (int64_t)(xcd + 1) * rows_per_xcd;
    if (r_end > rows_f1) r_end = rows_f1;
    const int64_t r_step = (int64_t)nj * G1_STAGE;

    floatx16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;

    constexpr int VCH = NT * 32 * G1_CPC;                // 16-byte chunks per staged V block
    constexpr int VQ = (VCH + 511) / 512;                // per thread (512 threads)
    uint4 vreg0[VQ], vreg1[VQ];
    uint4 areg0[G1_KS], areg1[G1_KS];

    auto load_v = [&](uint4 (&vreg)[VQ], int64_t r0) {
#pragma unroll
        for (int q = 0; q < VQ; ++q) {
            const int idx = tid + q * 512;
            if (idx >= VCH) continue;
            const int col = idx / G1_CPC, ch = idx % G1_CPC;
            const int64_t r = r0 + ch * 8;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (col < c && r < n) {
                const bf16_t* src = V + (int64_t)col * n + r;
                if (v_aligned && r + 8 <= n) {
                    val = *(const uint4*)src;
                } else {
                    u16x8 t;
#pragma unroll
                    for (int e = 0; e < 8; ++e) t.v[e] = (r + e < n) ? src[e].bits : (uint16_t)0;
                    val = __builtin_bit_cast(uint4, t);
                }
            }
            vreg[q] = val;
        }
    };
    auto store_v = [&](const uint4 (&vreg)[VQ], int64_t r0) {
#pragma unroll
        for (int q = 0; q < VQ; ++q) {
            const int idx = tid + q * 512;
            if (idx >= VCH) continue;
            const int col = idx / G1_CPC, ch = idx % G1_CPC;
            uint16_t* dst = Vs + col * VS_LD + ch * 8;
            if (!scaled) {
                *(uint4*)dst = vreg[q];
            } else {
                u16x8 raw = __builtin_bit_cast(u16x8, vreg[q]);
                u16x8 hi, lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int64_t r = r0 + ch * 8 + e;
                    const float hv = r < n ? h0[r] : 0.f;
                    const float prod = hv * bits_to_f32(raw.v[e]);
                    hi.v[e] = bf16_bits_rne(prod);
                    lo.v[e] = bf16_bits_rne(prod - bits_to_f32(hi.v[e]));
                }
                *(uint4*)dst = __builtin_bit_cast(uint4, hi);
                *(uint4*)(Vl + col * VS_LD + ch * 8) = __builtin_bit_cast(uint4, lo);
            }
        }
    };
    auto load_a = [&](uint4 (&areg)[G1_KS], int64_t r0) {
#pragma unroll
        for (int s = 0; s < G1_KS; ++s) {
            const int64_t rr = r0 + 16 * s;
            if (active && p < k && rr < r_end)
                areg[s] = *(const uint4*)(W + (rr / 16) * (int64_t)kmax * 16 + (int64_t)p * 16 + half * 8);
            else
                areg[s] = make_uint4(0, 0, 0, 0);
        }
    };

    if (r_begin < r_end) {
        load_v(vreg0, r_begin);
        load_a(areg0, r_begin);
    }
    if (r_begin + r_step < r_end) {
        load_v(vreg1, r_begin + r_step);
        load_a(areg1, r_begin + r_step);
    }
    auto stage = [&](uint4 (&vreg)[VQ], uint4 (&areg)[G1_KS], int64_t r0) {
        __syncthreads();
        store_v(vreg, r0);
        __syncthreads();
        if (r0 + 2 * r_step < r_end) load_v(vreg, r0 + 2 * r_step);
        if (active) {
#pragma unroll
            for (int s = 0; s < G1_KS; ++s) {
                const bf16x8 a = as_bf16x8(areg[s]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const uint16_t* bp = Vs + (t * 32 + (lane & 31)) * VS_LD + s * 16 + half * 8;
                    acc[t] = mfma32(a, as_bf16x8(*(const uint4*)bp), acc[t]);
                    if (scaled) {
                        const uint16_t* bl = Vl + (t * 32 + (lane & 31)) * VS_LD + s * 16 + half * 8;
                        acc[t] = mfma32(a, as_bf16x8(*(const uint4*)bl), acc[t]);
                    }
                }
            }
        }
        if (r0 + 2 * r_step < r_end) load_a(areg, r0 + 2 * r_step);
    };
    for (int64_t r0 = r_begin; r0 < r_end; r0 += 2 * r_step) {
        stage(vreg0, areg0, r0);
        if (r0 + r_step >= r_end) break;
        stage(vreg1, areg1, r0 + r_step);
    }
    if (!active) return;
    // partial Z for this row range: part[kr][col][2k], float32
    const int twok = 2 * k;
    float* dst = part + (int64_t)kr * twok * c;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 8 * (i / 4) + 4 * half + (i % 4);
            const int pp = wave * 32 + m;
            const int col = t * 32 + (lane & 31);
            if (pp < k && col < c) dst[(int64_t)col * twok + part_id * k + pp] = acc[t][i];
        }
    }
}

// Z (float64, column-major 2k x c) = fixed-order sum of the float32 partials;
// the Y rows are multiplied by gamma when B_0 = gamma I.
__global__ void reduce_z(int64_t count, int twok, int k, int nk, const float* __restrict__ part,
                         const double* __restrict__ scalars, int gamma_mode, double* __restrict__ Z) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= count) return;
    // eight interleaved partial sums in a fixed order keep eight loads in flight
    double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int q = 0;
    for (; q + 8 <= nk; q += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += (double)part[(int64_t)(q + u) * count + e];
    for (; q < nk; ++q) s8[0] += (double)part[(int64_t)q * count + e];
    double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    const int prow = (int)(e % twok);
    if (gamma_mode && prow >= k) s *= scalars[0];
    Z[e] = s;
}

// small^T (hi, lo): column j, position q of [Y phase (Gp*16) | S phase (Gp*16)]:
//   Y phase: -P(p, j), S phase: T(p, j), zero beyond k or c.
__global__ void pack_small(int k, int c, int cpad, int Gp, const double* __restrict__ P, const double* __restrict__ T,
                           uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
    const int K2 = 2 * Gp * 16;
    const int64_t total = (int64_t)cpad * K2;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / K2), q = (int)(e % K2);
        const int phase = q / (Gp * 16), pp = q % (Gp * 16);
        double v = 0.0;
        if (j < c && pp < k) v = phase == 0 ? -P[(int64_t)j * k + pp] : T[(int64_t)j * k + pp];
        const float vf = (float)v;
        const uint16_t h = bf16_bits_rne(vf);
        hi[e] = h;
        lo[e] = bf16_bits_rne((float)(v - (double)bits_to_f32(h)));
    }
}

// ---------------------------------------------------------------------------
// Pass 2: eight 32-row groups per workgroup (256 rows), MT2 column tiles.
// ---------------------------------------------------------------------------
constexpr int G2_ROWS = 256;
constexpr int SM_LD = 40;        // LDS pitch of a staged small column: 32 pairs + 8 pad
constexpr int G2_EP_LD = 264;    // LDS pitch (floats) of a staged output column: 256 rows + 8 pad

// Up to four column tiles one wave per 32-row group holds them all (8 waves).  From
// five tiles two waves share each row group (SPLIT = 2), each owning MH of the MT2
// tiles: the W fragments are read by both (the second read hits in cache), and the
// halved accumulator set lets four waves share a SIMD.  Measured on the full grid: one
// wave per row group is 14 % faster for two to four tiles, two are 6 % faster for five
// and 10 % faster for seven.
template <int MT2>
struct G2Shape {
    static constexpr int SPLIT = MT2 > 4 ? 2 : 1;
    static constexpr int MH = (MT2 + SPLIT - 1) / SPLIT;
    static constexpr int THREADS = 64 * (G2_ROWS / 32) * SPLIT;
};

template <int MT2, bool DIFF>
__global__ void __launch_bounds__(G2Shape<MT2>::THREADS) gemm2_mfma(int64_t n, int c, int G, int Gp,
                                                                   const bf16_t* __restrict__ Y2,
                                                                   const bf16_t* __restrict__ S2,
                                                                   const uint16_t* __restrict__ shi,
                                                                   const uint16_t* __restrict__ slo,
                                                                   const float* __restrict__ h0,
                                                                   const bf16_t* __restrict__ V, float* __restrict__ out) {
    constexpr int SPLIT = G2Shape<MT2>::SPLIT, MH = G2Shape<MT2>::MH, NTH = G2Shape<MT2>::THREADS;
    // LDS: two buffers of the staged small operand (hi, lo), [col][SM_LD]
    extern __shared__ unsigned char smem_raw[];
    constexpr int BUF = MT2 * 32 * SM_LD;
    uint16_t* sm = (uint16_t*)smem_raw;   // buffer b: hi at sm + 2*b*BUF, lo at sm + (2*b+1)*BUF
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, half = lane >> 5;
    // row group and column share; the share alternates between waves 4 apart, which
    // sit on the same SIMD, so every SIMD gets one wave of each share
    const int rg = wave / SPLIT, cs = SPLIT == 2 ? ((wave ^ (wave >> 2)) & 1) : 0;
    const int mt0 = cs * MH;                               // first column tile of this wave
    const int ntw = min(MH, MT2 - mt0);                    // tiles of this wave (uniform)
    // Row block: workgroup g runs on XCD g % 8, and each XCD walks a contiguous eighth
    // of the row blocks in order, so the column-major V reads and output writes of the
    // workgroups an XCD runs at once form long runs per column.
    const int nblk = (int)((n + G2_ROWS - 1) / G2_ROWS), per_xcd = (nblk + 7) / 8;
    const int blk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (blk >= nblk) return;                              // whole workgroup
    const int64_t row_base = (int64_t)blk * G2_ROWS + rg * 32;
    const int64_t rb32 = row_base / 32;
    const int K2 = 2 * Gp * 16;
    const int nchunks = K2 / 32;
    const bool row_ok = row_base + (lane & 31) < n;
    const float h0r = row_ok ? h0[row_base + (lane & 31)] : 0.f;

    floatx16 acc[MH];
#pragma unroll
    for (int t = 0; t < MH; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;

    constexpr int SCH = MT2 * 32 * 4;        // 16-byte chunks of one array per staged chunk (<= 1024)
    static_assert(SCH <= 1024, "one staging chunk per thread and array");
    uint4 sh0 = make_uint4(0, 0, 0, 0), sl0 = sh0, sh1 = sh0, sl1 = sh0;
#define G2_LOAD_SMALL(T)                                                        \
    {                                                                           \
        if (tid < SCH) {                                                        \
            const int64_t off = (int64_t)(tid >> 2) * K2 + (T) * 32 + (tid & 3) * 8; \
            sh0 = *(const uint4*)(shi + off);                                   \
            sl0 = *(const uint4*)(slo + off);                                   \
        }                                                                       \
        if (NTH < SCH && tid + NTH < SCH) {                                     \
            const int64_t off = (int64_t)((tid + NTH) >> 2) * K2 + (T) * 32 + (tid & 3) * 8; \
            sh1 = *(const uint4*)(shi + off);                                   \
            sl1 = *(const uint4*)(slo + off);                                   \
        }                                                                       \
    }
#define G2_STORE_SMALL(B)                                                                   \
    {                                                                                       \
        uint16_t* H_ = sm + 2 * (B) * BUF;                                                  \
        uint16_t* L_ = H_ + BUF;                                                            \
        if (tid < SCH) {                                                                    \
            *(uint4*)(H_ + (tid >> 2) * SM_LD + (tid & 3) * 8) = sh0;                       \
            *(uint4*)(L_ + (tid >> 2) * SM_LD + (tid & 3) * 8) = sl0;                       \
        }                                                                                   \
        if (NTH < SCH && tid + NTH < SCH) {                                                 \
            *(uint4*)(H_ + ((tid + NTH) >> 2) * SM_LD + (tid & 3) * 8) = sh1;               \
            *(uint4*)(L_ + ((tid + NTH) >> 2) * SM_LD + (tid & 3) * 8) = sl1;               \
        }                                                                                   \
    }
    // Every call issues a load: a chunk past the end re-reads the last chunk (unused), and a
    // padding group past G re-reads group G - 1, whose product with the zero rows of the
    // small operand is exactly zero.  With no branch or select on the result, each prefetch
    // slot stays in one register set and the loop carries no copies (nor the wait for all
    // outstanding loads that such copies would force at the back edge).
    auto load_b = [&](int t, int sg) -> uint4 {
        const int gq = 2 * min(t, nchunks - 1) + sg;
        const int phase = gq >= Gp ? 1 : 0;
        const int grp = min(gq - phase * Gp, G - 1);
        const bf16_t* W = phase ? S2 : Y2;
        return *(const uint4*)(W + rb32 * (int64_t)G * 512 + (int64_t)grp * 512 + (lane & 31) * 16 + half * 8);
    };

    // W fragments run DEPTH chunks ahead of the MFMAs.
    constexpr int DEPTH = MH >= 4 ? 2 : 4;
    uint4 bq0[DEPTH], bq1[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
        bq0[d] = load_b(d, 0);
        bq1[d] = load_b(d, 1);
    }
    G2_LOAD_SMALL(0)
    G2_STORE_SMALL(0)
    G2_LOAD_SMALL(min(1, nchunks - 1))
    __syncthreads();
    for (int t0 = 0; t0 < nchunks; t0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int t = t0 + d;
            // The loads run unconditionally (clamped chunk indices) so that the prefetch
            // registers take the same path on every iteration; only the LDS store and the
            // MFMAs are skipped for a chunk past the end.
            const int buf = t & 1;
            if (t + 1 < nchunks) G2_STORE_SMALL(buf ^ 1)
            G2_LOAD_SMALL(min(t + 2, nchunks - 1))
            const uint16_t* H = sm + 2 * buf * BUF;
            const uint16_t* L = H + BUF;
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                if (t < nchunks) {
                    const bf16x8 b = as_bf16x8(sg ? bq1[d] : bq0[d]);
#pragma unroll
                    for (int m = 0; m < MH; ++m) {
                        if (m < ntw) {
                            const int off = ((mt0 + m) * 32 + (lane & 31)) * SM_LD + sg * 16 + half * 8;
                            acc[m] = mfma32(as_bf16x8(*(const uint4*)(H + off)), b, acc[m]);
                            acc[m] = mfma32(as_bf16x8(*(const uint4*)(L + off)), b, acc[m]);
                        }
                    }
                }
                // refill the slot just consumed: its register is free once the MFMAs
                // above have read it, so the loop needs no register copies
                if (sg) bq1[d] = load_b(t + DEPTH, 1);
                else bq0[d] = load_b(t + DEPTH, 0);
            }
            if (t < nchunks) {
                if (2 * t + 2 == Gp) {
                    // end of the Y phase: acc holds -(Y P)^T for this lane's row; scale by h0[row]
#pragma unroll
                    for (int m = 0; m < MH; ++m)
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[m][i] *= h0r;
                }
                __syncthreads();
            }
        }
    }
#undef G2_LOAD_SMALL
#undef G2_STORE_SMALL
    // Output through LDS.  Pass p stages column tile p of each column share as
    // [column][row] (256 rows per column), then every wave writes four whole columns:
    // lane l covers rows 4l .. 4l+3 of the workgroup, so each column is one contiguous
    // 1 KB store (16 bytes per lane) and its V rows one contiguous 512-byte load.  The
    // small-operand buffers are free by now (last barrier of the loop).
    float* ep = (float*)smem_raw;                        // [SPLIT * 32][G2_EP_LD]
    const int64_t r4 = (int64_t)blk * G2_ROWS + lane * 4;
    const bool vec = (n % 4) == 0 && (((uintptr_t)out) & 15) == 0 && (DIFF || (((uintptr_t)V) & 7) == 0);
    float h4[4] = {0.f, 0.f, 0.f, 0.f};
    if (!DIFF) {
#pragma unroll
        for (int e = 0; e < 4; ++e) h4[e] = r4 + e < n ? h0[r4 + e] : 0.f;
    }
#pragma unroll
    for (int p = 0; p < MH; ++p) {
        // V rows of this pass's four columns, issued before the staging barrier
        uint2 vq[4];
        if (!DIFF) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = wave * 4 + j, qs = q / 32, col = (qs * MH + p) * 32 + q % 32;
                vq[j] = make_uint2(0, 0);
                const bool has = p < min(MH, MT2 - qs * MH) && col < c;
                if (has && vec && r4 + 4 <= n) vq[j] = *(const uint2*)(V + (int64_t)col * n + r4);
            }
        }
        if (p < ntw) {
            float* dst = ep + cs * 32 * G2_EP_LD + rg * 32 + (lane & 31);
#pragma unroll
            for (int i = 0; i < 16; ++i) dst[(8 * (i / 4) + 4 * half + (i % 4)) * G2_EP_LD] = acc[p][i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = wave * 4 + j, qs = q / 32, col = (qs * MH + p) * 32 + q % 32;
            if (p >= min(MH, MT2 - qs * MH) || col >= c) continue;
            const float4 a = *(const float4*)(ep + q * G2_EP_LD + lane * 4);
            float o[4] = {a.x, a.y, a.z, a.w};
            float* dst = out + (int64_t)col * n + r4;
            if (vec && r4 + 4 <= n) {
                if (!DIFF) {
                    o[0] += h4[0] * bits_to_f32((uint16_t)(vq[j].x & 0xffffu));
                    o[1] += h4[1] * bits_to_f32((uint16_t)(vq[j].x >> 16));
                    o[2] += h4[2] * bits_to_f32((uint16_t)(vq[j].y & 0xffffu));
                    o[3] += h4[3] * bits_to_f32((uint16_t)(vq[j].y >> 16));
                }
                *(float4*)dst = make_float4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (r4 + e >= n) break;
                    float v = o[e];
                    if (!DIFF) v += h4[e] * bits_to_f32(V[(int64_t)col * n + r4 + e].bits);
                    dst[e] = v;
                }
            }
        }
        __syncthreads();
    }
}

template <int NT, bool DIAG>
void launch_g1(int grid, int threads, size_t smem, hipStream_t st, int64_t n, int k, int kmax, int c, const bf16_t* S1,
               const bf16_t* Y1, const float* h0, const bf16_t* V, float* part, int64_t rows_per_wg, int64_t rows_f1,
               int nk, int aligned) {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)gemm1_mfma<NT, DIAG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  2 * 8 * 32 * G1Shape<NT>::LD * (int)sizeof(uint16_t));
        attr = true;
    }
    hipLaunchKernelGGL((gemm1_mfma<NT, DIAG>), dim3(grid), dim3(threads), smem, st, n, k, kmax, c, S1, Y1, h0, V, part,
                       rows_per_wg, rows_f1, nk, aligned);
}

typedef void (*g1_fn)(int, int, size_t, hipStream_t, int64_t, int, int, int, const bf16_t*, const bf16_t*, const float*,
                      const bf16_t*, float*, int64_t, int64_t, int, int);

g1_fn pick_g1(int NT, bool diag) {
#define G1CASE(N)                                        \
    case N:                                              \
        return diag ? launch_g1<N, true> : launch_g1<N, false>;
    switch (NT) {
        G1CASE(1) G1CASE(2) G1CASE(3) G1CASE(4) G1CASE(5) G1CASE(6) G1CASE(7) G1CASE(8)
    }
#undef G1CASE
    return nullptr;
}

template <int MT2, bool DIFF>
void launch_g2(int grid, hipStream_t st, int64_t n, int c, int G, int Gp, const bf16_t* Y2, const bf16_t* S2,
               const uint16_t* shi, const uint16_t* slo, const float* h0, const bf16_t* V, float* out) {
    // small-operand double buffer, reused by the epilogue for SPLIT x 32 output columns
    constexpr int NTH = G2Shape<MT2>::THREADS;
    const size_t smem = std::max((size_t)4 * MT2 * 32 * SM_LD * sizeof(uint16_t),
                                 (size_t)G2Shape<MT2>::SPLIT * 32 * G2_EP_LD * sizeof(float));
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)gemm2_mfma<MT2, DIFF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem);
        attr = true;
    }
    hipLaunchKernelGGL((gemm2_mfma<MT2, DIFF>), dim3(grid), dim3(NTH), smem, st, n, c, G, Gp, Y2, S2, shi, slo, h0, V,
                       out);
}

typedef void (*g2_fn)(int, hipStream_t, int64_t, int, int, int, const bf16_t*, const bf16_t*, const uint16_t*,
                      const uint16_t*, const float*, const bf16_t*, float*);

g2_fn pick_g2(int MT2, bool diff) {
#define G2CASE(N)                                        \
    case N:                                              \
        return diff ? launch_g2<N, true> : launch_g2<N, false>;
    switch (MT2) {
        G2CASE(1) G2CASE(2) G2CASE(3) G2CASE(4) G2CASE(5) G2CASE(6) G2CASE(7) G2CASE(8)
    }
#undef G2CASE
    return nullptr;
}

}  // namespace

// Layout sizes shared with the runtime.
int64_t mfma_rows_f1(int64_t n) { return round_up(n, 64); }
int64_t mfma_rows_f2(int64_t n) { return round_up(n, 256); }
int mfma_groups(int kmax) { return (kmax + 15) / 16; }

int mfma_scatter_pair(bfgsuq_ctx* h, int j) {
    const int G = mfma_groups(h->kmax);
    const int64_t r1 = mfma_rows_f1(h->n), r2 = mfma_rows_f2(h->n);
    const int64_t rows = r1 > r2 ? r1 : r2;
    const int grid = (int)std::min<int64_t>(4096, (rows + 255) / 256);
    hipLaunchKernelGGL(scatter_pair_layouts, dim3(grid), dim3(256), 0, h->stream, h->n, r1, r2, h->kmax, G, j,
                       (const bf16_t*)h->S + (int64_t)j * h->ld, (const bf16_t*)h->Y + (int64_t)j * h->ld,
                       (bf16_t*)h->S1, (bf16_t*)h->Y1, (bf16_t*)h->S2, (bf16_t*)h->Y2);
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

bool mfma_apply_supported(const bfgsuq_ctx* h, int c) {
    return h->storage == BFGS_BF16 && h->S1 != nullptr && h->k >= 1 && h->k <= 256 && c >= 1 && c <= 256;
}

int apply_small_solve(bfgsuq_ctx* h, int c, const double* Z, double* P, double* T);

size_t apply_small16_bytes(int kmax) { return (size_t)2 * 256 * 2 * (mfma_groups(kmax) + 1) * 16 * 2; }

int mfma_apply(bfgsuq_ctx* h, const void* Vv, int c, void* outv, bool diff, const ApplyWs* fixed) {
    const int64_t n = h->n;
    const int k = h->k;
    const bf16_t* V = (const bf16_t*)Vv;
    float* out = (float*)outv;
    const int NT = (c + 31) / 32;
    int nk = std::max(8, (h->g1_nk + 7) / 8 * 8);         // row slots, 1/8 per XCD (tunable)
    const int64_t rows_f1 = mfma_rows_f1(n);
    const int64_t rows_per_xcd = round_up((rows_f1 + 7) / 8, g1_stage(NT));
    const int twok = 2 * k;
    const int G = mfma_groups(h->kmax);
    const int Gk = (k + 15) / 16;                          // groups that hold pairs
    const int Gp = (Gk + 1) / 2 * 2;
    const int cpad = NT * 32;
    int rc;
    float* part;
    double *Z, *P;
    uint16_t* shi;
    const size_t slot_bytes = (size_t)twok * c * sizeof(float);
    if (fixed) {
        const int cap = (int)(fixed->part_bytes / slot_bytes) / 8 * 8;
        if (cap < 8) return BFGS_ERR_ARG;
        nk = std::min(nk, cap);
        part = (float*)fixed->part;
        Z = fixed->Z;
        P = fixed->PT;
        shi = fixed->small16;
    } else {
        if ((rc = ensure_ws(h->part, (size_t)nk * slot_bytes)) != BFGS_OK) return rc;
        if ((rc = ensure_ws(h->Z, (size_t)2 * h->kmax * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
        if ((rc = ensure_ws(h->PT, (size_t)2 * h->kmax * BFGS_MAX_COLS * 8)) != BFGS_OK) return rc;
        if ((rc = ensure_ws(h->small16, apply_small16_bytes(h->kmax))) != BFGS_OK) return rc;
        part = (float*)h->part.ptr;
        Z = (double*)h->Z.ptr;
        P = (double*)h->PT.ptr;
        shi = (uint16_t*)h->small16.ptr;
    }
    double* T = P + (size_t)k * c;
    uint16_t* slo = shi + (size_t)cpad * 2 * Gp * 16;
    const bool diag = !h->gamma_mode;
    {
        ProfScope ps(h, diff ? "hdiff_gemm1" : "apply_gemm1");
        const size_t smem = (size_t)(diag ? 2 : 1) * NT * 32 * (g1_stage(NT) + 8) * sizeof(uint16_t);
        const int grid = 2 * nk;                           // S and Y workgroup per slot
        const int aligned = (n % 8 == 0) && (((uintptr_t)V) % 16 == 0);
        pick_g1(NT, diag)(grid, 512, smem, h->stream, n, k, h->kmax, c, (const bf16_t*)h->S1,
                          (const bf16_t*)h->Y1, (const float*)h->h0, V, part, rows_per_xcd, rows_f1, nk, aligned);
    }
    {
        ProfScope ps(h, "apply_reduce");
        const int64_t count = (int64_t)twok * c;
        hipLaunchKernelGGL(reduce_z, dim3(ceil_div(count, 256)), dim3(256), 0, h->stream, count, twok, k, nk, part,
                           h->scalars, h->gamma_mode ? 1 : 0, Z);
    }
    if ((rc = apply_small_solve(h, c, Z, P, T)) != BFGS_OK) return rc;
    {
        ProfScope ps(h, "apply_pack");
        const int64_t total = (int64_t)cpad * 2 * Gp * 16;
        hipLaunchKernelGGL(pack_small, dim3((int)std::min<int64_t>(2048, (total + 255) / 256)), dim3(256), 0, h->stream,
                           k, c, cpad, Gp, P, T, shi, slo);
    }
    {
        ProfScope ps(h, diff ? "hdiff_gemm2" : "apply_gemm2");
        const int grid = 8 * ceil_div(ceil_div(n, G2_ROWS), 8);   // whole number of blocks per XCD
        pick_g2(NT, diff)(grid, h->stream, n, c, G, Gp, (const bf16_t*)h->Y2, (const bf16_t*)h->S2, shi, slo,
                          (const float*)h->h0, V, out);
    }
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}
