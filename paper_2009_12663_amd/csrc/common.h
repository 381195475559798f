// Internal definitions shared by the HIP sources of libbfgsuq (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "../../include/bfgsuq.h"

// ---------------------------------------------------------------------------
// Storage types.  bf16_t is the raw bit pattern of a bfloat16.
// ---------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(bf16_t h) {
    union { uint32_t u; float f; } v;
    v.u = ((uint32_t)h.bits) << 16;
    return v.f;
}

// Round-to-nearest-even float -> bfloat16; NaN stays NaN (quiet).
__host__ __device__ inline bf16_t float_to_bf16(float f) {
    union { uint32_t u; float f; } v;
    v.f = f;
    uint32_t u = v.u;
    bf16_t out;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        out.bits = (uint16_t)((u >> 16) | 0x40u);
        return out;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    out.bits = (uint16_t)(u >> 16);
    return out;
}

template <typename T> struct DT;
template <> struct DT<double> { static constexpr bfgs_dtype code = BFGS_F64; };
template <> struct DT<float> { static constexpr bfgs_dtype code = BFGS_F32; };
template <> struct DT<bf16_t> { static constexpr bfgs_dtype code = BFGS_BF16; };

__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(float x) { return (double)x; }
__device__ __forceinline__ double to_f64(bf16_t x) { return (double)bf16_to_float(x); }
__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(bf16_t x) { return bf16_to_float(x); }
__device__ __forceinline__ float to_f32(double x) { return (float)x; }

template <typename T> __device__ __forceinline__ T from_f64(double x);
template <> __device__ __forceinline__ double from_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_f64<float>(double x) { return (float)x; }
// float64 -> float32 -> bfloat16, each to nearest-even.
template <> __device__ __forceinline__ bf16_t from_f64<bf16_t>(double x) { return float_to_bf16((float)x); }

// float64 -> bfloat16 with a single rounding to nearest-even: the float64 value is
// first rounded to float32 by round-to-odd (truncate, then set the last bit if
// anything was cut off), which keeps every bit that decides the final rounding
// because float32 carries 16 more significant bits than bfloat16 (round-to-odd to
// at least p + 2 bits followed by round-to-nearest to p bits is exact).
__device__ __forceinline__ bf16_t f64_to_bf16_rne(double x) {
    float f = (float)x;
    const double back = (double)f;
    if (back != x && x == x) {
        uint32_t u = __builtin_bit_cast(uint32_t, f);
        if (fabs(back) > fabs(x)) u -= 1u;   // rounded away from zero: step back to the truncation
        u |= 1u;
        f = __builtin_bit_cast(float, u);
    }
    return float_to_bf16(f);
}

template <typename T> __device__ __forceinline__ T from_f32(float x);
template <> __device__ __forceinline__ float from_f32<float>(float x) { return x; }
template <> __device__ __forceinline__ double from_f32<double>(float x) { return (double)x; }
template <> __device__ __forceinline__ bf16_t from_f32<bf16_t>(float x) { return float_to_bf16(x); }

inline size_t dtype_size(bfgs_dtype d) { return d == BFGS_F64 ? 8 : d == BFGS_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------
// Handle.
// ---------------------------------------------------------------------------
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    unsigned gen = 0;          // bumped on every (re)allocation: captured graphs hold ptr
};

// Optional per-kernel timing with HIP events on the handle's stream.
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
    bool ended = false;
};

// Stage timers: begin/end pairs may nest (an end closes the innermost open stage).
struct Profiler {
    bool on = false;
    std::vector<ProfRec> recs;
    std::vector<size_t> open;   // indices into recs of the stages not yet ended
    std::vector<hipEvent_t> pool;
    size_t used = 0;
};

struct bfgsuq_ctx {
    int64_t n = 0;
    int64_t ld = 0;            // leading dimension of S and Y (n rounded up to 128)
    int32_t kmax = 0;
    int32_t k = 0;
    bfgs_dtype storage = BFGS_F32;
    bool gamma_mode = false;   // B_0 = gamma I, gamma from the first pair
    bool gamma_known = false;
    hipStream_t stream = nullptr;

    void* S = nullptr;         // ld x kmax, column-major, storage type
    void* Y = nullptr;
    void* h0 = nullptr;        // n, storage-real type (double for F64, float otherwise)
    double* Rm = nullptr;      // kmax x kmax column-major: Rm[j*kmax + i] = s_i^T y_j
    double* YHY = nullptr;     // kmax x kmax symmetric: y_i^T B_0 y_j
    double* Rinv = nullptr;    // kmax x kmax column-major: inverse of the upper triangle of Rm
    double* RinvT = nullptr;   // its transpose, column-major (RinvT[l * kmax + i] = Rinv(l, i))
    double* gram_part = nullptr;   // partial sums for push
    double* scalars = nullptr; // [0] = gamma, [1] = last s^T y, [2] = last y^T y
    int32_t* status = nullptr; // deferred device status (0 = OK)
    int gram_blocks = 0;

    // bfloat16 MFMA layouts of S and Y (see apply_mfma.hip); null for other storage types
    void* S1 = nullptr;
    void* Y1 = nullptr;
    void* S2 = nullptr;
    void* Y2 = nullptr;

    // apply workspaces (grow-only)
    Workspace part, Z, PT, small16;
    // rsvd workspaces
    Workspace X, E, Q, W, refl, tau, Rtree, small, lam, diag;
    int32_t last_rank = 0;
    bool have_rsvd = false;
    // tunables (bfgs_autotune): row ranges of the pass-1 MFMA kernel, TSQR chains (power of two)
    int g1_nk = 128;
    int qr_chains = 256;
    // bumped whenever k or a tunable changes; with the workspaces' counters it tells a
    // captured graph (which holds k, the tunables and the workspace pointers) that it
    // no longer matches the handle
    unsigned gen = 0;
    double* host_sc = nullptr; // pinned host copy of scalars for push_pair's check
    Profiler prof;

    // Out-of-core history (bfgs_create_streamed): S and Y in pinned host memory (same
    // layout), staged to the device in row slices of slice_rows through two buffers
    // (leading dimension slice_ld) by a copy stream, so that the copy of one slice
    // overlaps the kernels of the previous one.
    bool streamed = false;
    int64_t slice_rows = 0, slice_ld = 0;
    void* stage[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [buffer][S, Y]
    void* push_tmp = nullptr;  // the pair being pushed, rounded to storage (2 x n)
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr}, ev_start = nullptr;
};

// Streams the first ncols columns of S and Y through the staging buffers, one row
// slice at a time, and calls body(slice, r0, rows, S_slice, Y_slice) for each once its
// copy has landed (body enqueues on the handle's stream; the slices' columns are
// slice_ld apart).
int stream_slices(bfgsuq_ctx* h, int ncols,
                  const std::function<int(int, int64_t, int64_t, const void*, const void*)>& body);

// Sum of the counters a captured graph depends on.
inline unsigned long long handle_generation(const bfgsuq_ctx* h) {
    const Workspace* ws[] = {&h->part, &h->Z, &h->PT, &h->small16, &h->X, &h->E, &h->Q, &h->W, &h->refl, &h->tau,
                             &h->Rtree, &h->small, &h->lam, &h->diag};
    unsigned long long g = h->gen;
    for (const Workspace* w : ws) g += w->gen;
    return g;
}

void prof_begin(bfgsuq_ctx* h, const char* name);
void prof_end(bfgsuq_ctx* h);

// Scoped helper: times the launches issued while it lives.
struct ProfScope {
    bfgsuq_ctx* h;
    ProfScope(bfgsuq_ctx* hh, const char* name) : h(hh) { prof_begin(h, name); }
    ~ProfScope() { prof_end(h); }
};

#define BFGS_HIP(expr)                                  \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return BFGS_ERR_HIP;      \
    } while (0)

int ensure_ws(Workspace& w, size_t bytes);

// Deferred status codes written by kernels (plain stores, no atomics).
__device__ __forceinline__ void set_status(int32_t* status, int32_t code) {
    if (status[0] == 0) status[0] = code;
}

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Entry points implemented in the other translation units.
// ---------------------------------------------------------------------------
// Scratch of one apply call: the split-K partials of pass 1, Z (2k x c float64),
// P and T (k x c float64 each) and the bfloat16 hi/lo small operand of pass 2.
// apply_block grows them in the handle's workspaces unless it is given a fixed
// buffer (the allocation-free entry point); with a fixed buffer the split-K depth
// is capped so that the partials fit in part_bytes.
struct ApplyWs {
    void* part = nullptr;
    size_t part_bytes = 0;
    double* Z = nullptr;        // >= 2 * k_max * BFGS_MAX_COLS doubles
    double* PT = nullptr;       // >= 2 * k_max * BFGS_MAX_COLS doubles
    uint16_t* small16 = nullptr;// >= apply_small16_bytes(k_max)
};
size_t apply_small16_bytes(int kmax);

// out is float64 when out64 (float32 storage only: the rSVD keeps E in float64), else
// the storage's result type.
int apply_block(bfgsuq_ctx* h, const void* V, int32_t ncols, void* out, bool diff, bool out64 = false,
                const ApplyWs* fixed = nullptr);
// (B_k - B_0) V for a float32 or float64 block (float64 matrix cores, any storage);
// out float64 or float32.
int apply_diff_float_block(bfgsuq_ctx* h, const void* V, bool v64, int32_t ncols, void* out, bool out64);
// rSVD variants (flags of bfgs_rsvd_ex)
int rsvd_run(bfgsuq_ctx* h, int32_t rank, int32_t oversample, uint64_t seed, void* U, double* Sigma,
             uint32_t flags = 0);
// Blocked Householder TSQR E = Q R (E column-major n x c; *R_out: row-major c x c in
// the handle's workspace).  tsqr.hip.  E's rows are split into chains of
// tsqr_chain_rows(h) rows (a multiple of QR_TILE; *nchains of them, the last ones
// possibly short or empty).  Q is column-major n x c, or with q_blocked chain-blocked:
// row r of column j at (r / B) B c + j B + r % B for B = tsqr_chain_rows(h), so each
// chain's rows of Q are one contiguous block (ceil(n / B) B c elements in all).
constexpr int QR_TILE = 64;
int64_t tsqr_chain_rows(const bfgsuq_ctx* h, int* nchains = nullptr);
int tsqr_run(bfgsuq_ctx* h, int c, const float* E, float* Q, double** R_out, bool q_blocked = false);
int tsqr_run(bfgsuq_ctx* h, int c, const double* E, float* Q, double** R_out);
int tsqr_run(bfgsuq_ctx* h, int c, const double* E, double* Q, double** R_out);
// Whether the TSQR of a c-column block keeps its per-chain triangle in float64.
bool tsqr_f64_slot(int c);
// Eigenpairs of the symmetric tridiagonal (d, e), c <= 256, by divide and conquer:
// *w_out -> the eigenvalues (in work), Z = Qh Y with Y their eigenvectors (c x c
// column-major device arrays); work holds tridiag_dc_workspace(c) bytes.
size_t tridiag_dc_workspace(int c);
// bfloat16-storage forms of the rSVD's tall products (rsvd_bf16.hip): Q^T X chunk
// partials (float64, the layout qtx_mfma writes), and the basis U = Q Us[:, :rank]
// with the posterior diagonal dout = h0 + sum_j lam_j U_j^2; ush holds
// basis_bf16_workspace(c, rank) bytes of split Us.  q_block: 0 for a column-major Q,
// else the block rows B of a chain-blocked Q (tsqr_run); for qtx the chunks are then
// the blocks (rows_per_chunk == q_block).
int qtx_bf16_launch(hipStream_t st, int64_t n, int c, const float* Q, const bf16_t* X, double* part, int nchunks,
                    int64_t rows_per_chunk, int64_t q_block = 0);
size_t basis_bf16_workspace(int c, int rank);
int basis_bf16_launch(hipStream_t st, int64_t n, int c, int rank, const float* Q, const double* Us, uint16_t* ush,
                      const double* lam, const float* h0, float* U, float* dout, int32_t* status,
                      bool whitened = false, int64_t q_block = 0);
int tridiag_dc(hipStream_t st, int c, const double* d, const double* e, const double* Qh, double* work, double** w_out,
               double* Z, int32_t* status);
int probes_run(bfgsuq_ctx* h, uint64_t seed, int32_t ncols, void* X);
int64_t mfma_rows_f1(int64_t n);
int64_t mfma_rows_f2(int64_t n);
int mfma_groups(int kmax);
int mfma_scatter_pair(bfgsuq_ctx* h, int j);
bool mfma_apply_supported(const bfgsuq_ctx* h, int c);
int mfma_apply(bfgsuq_ctx* h, const void* V, int c, void* out, bool diff, const ApplyWs* fixed);
int apply_small_solve(bfgsuq_ctx* h, int c, const double* Z, double* P, double* T);

// One problem of a persistent batched apply (device copy read by the pass kernels).
struct PersistProblem {
    int64_t n, ld, rows_per_chunk;
    int k, kmax, c, ptiles, ctiles, nchunks, first1, first2;
    const void *S, *Y, *h0, *V;
    void* out;
    double *part, *Z, *P;
    const double *Rm, *Rinv, *RinvT, *YHY;
    int32_t* status;
};

// Device descriptors and work-queue heads of one persistent batched apply (a batch
// keeps one for eager calls and one for its captured graph).
struct PersistSlot {
    PersistProblem* prob = nullptr;
    size_t cap = 0;
    unsigned* head = nullptr;
    int nprob = 0, items1 = 0, items2 = 0, solve_blocks = 0;
};

// Apply B_k of every problem to its block (float32 or float64 storage, all of one
// type, 1 <= k <= 256): four launches on st in all (queue reset, pass 1 of every
// problem, the small solves, pass 2).  upload = false reuses the slot's descriptors
// (a graph capture after an eager call with the same arguments).  wg_per_cu sets the
// persistent grid (workgroups per compute unit).
int batch_apply_persistent(bfgsuq_ctx* const* hs, int nprob, const void* const* V, const int32_t* ncols,
                           void* const* out, hipStream_t st, PersistSlot* slot, bool upload, int wg_per_cu);
int push_enqueue(bfgsuq_ctx* h, const void* s, const void* y, bfgs_dtype in_dtype);
int push_finish(bfgsuq_ctx* h);
// Forget the oldest pair (float32/float64 storage, device-resident history).
int pop_oldest(bfgsuq_ctx* h);
