// Handle life cycle, pair storage and the k x k matrices of the compact form.
//
// The inverse BFGS matrix of eq. (3) after k pairs is kept implicitly: the
// pairs themselves (column-major S, Y in HBM, in the storage type) plus two
// k x k float64 matrices built from the *stored* values as pairs arrive,
//   Rm(i, j)  = s_i^T y_j   (upper triangle i <= j is the R of the compact form,
//                            its diagonal the curvatures 1 / r_i of Alg. 1)
//   YHY(i, j) = y_i^T B_0 y_j
// Pushing pair j costs one pass over the j + 1 stored columns (O(n j)).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "common.h"

int ensure_ws(Workspace& w, size_t bytes) {
    if (bytes <= w.bytes) return BFGS_OK;
    if (w.ptr) {
        if (hipFree(w.ptr) != hipSuccess) return BFGS_ERR_HIP;
        w.ptr = nullptr;
        w.bytes = 0;
    }
    ++w.gen;
    if (hipMalloc(&w.ptr, bytes) != hipSuccess) {
        w.ptr = nullptr;
        return BFGS_ERR_ALLOC;
    }
    w.bytes = bytes;
    return BFGS_OK;
}

static hipEvent_t prof_event(bfgsuq_ctx* h) {
    Profiler& P = h->prof;
    if (P.used == P.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        P.pool.push_back(e);
    }
    return P.pool[P.used++];
}

void prof_begin(bfgsuq_ctx* h, const char* name) {
    if (!h->prof.on) return;
    ProfRec r;
    r.name = name;
    r.a = prof_event(h);
    r.b = prof_event(h);
    if (!r.a || !r.b) return;
    if (hipEventRecord(r.a, h->stream) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    h->prof.open.push_back(h->prof.recs.size());
    h->prof.recs.push_back(r);
}

void prof_end(bfgsuq_ctx* h) {
    if (!h->prof.on || h->prof.open.empty()) return;
    ProfRec& r = h->prof.recs[h->prof.open.back()];
    h->prof.open.pop_back();
    if (hipEventRecord(r.b, h->stream) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    r.ended = true;
}

static void free_ws(Workspace& w) {
    if (w.ptr) (void)hipFree(w.ptr);
    w.ptr = nullptr;
    w.bytes = 0;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <typename Tin, typename Tst>
__global__ void store_pair_kernel(int64_t n, const Tin* __restrict__ s, const Tin* __restrict__ y,
                                  Tst* __restrict__ Scol, Tst* __restrict__ Ycol) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        Scol[r] = from_f64<Tst>(to_f64(s[r]));
        Ycol[r] = from_f64<Tst>(to_f64(y[r]));
    }
}

// float64 input to bfloat16 storage: one rounding to nearest-even.
template <>
__global__ void store_pair_kernel<double, bf16_t>(int64_t n, const double* __restrict__ s,
                                                  const double* __restrict__ y, bf16_t* __restrict__ Scol,
                                                  bf16_t* __restrict__ Ycol) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        Scol[r] = f64_to_bf16_rne(s[r]);
        Ycol[r] = f64_to_bf16_rne(y[r]);
    }
}

// float32 input to bfloat16 storage: one rounding (float32 -> bfloat16).
template <>
__global__ void store_pair_kernel<float, bf16_t>(int64_t n, const float* __restrict__ s,
                                                 const float* __restrict__ y, bf16_t* __restrict__ Scol,
                                                 bf16_t* __restrict__ Ycol) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        Scol[r] = float_to_bf16(s[r]);
        Ycol[r] = float_to_bf16(y[r]);
    }
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Partial sums over row chunk b of s_i^T y_j and y_i^T (h0 o y_j) (or y_i^T y_j
// when B_0 = gamma I), for i = blockIdx.y, stored as partial b0 + b of nbt per i (a
// history streamed in row slices fills its partials one slice at a time).
template <typename Tst, typename Th>
__global__ void __launch_bounds__(256) gram_partial_kernel(int64_t n, int64_t ld, int j, const Tst* __restrict__ S,
                                                           const Tst* __restrict__ Y, const Th* __restrict__ h0,
                                                           int gamma_mode, double* __restrict__ part, int b0, int nbt) {
    __shared__ double sh[8];
    const int i = blockIdx.y, b = blockIdx.x, nb = gridDim.x;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t r0 = b * chunk, r1 = min(n, r0 + chunk);
    const Tst* si = S + (int64_t)i * ld;
    const Tst* yi = Y + (int64_t)i * ld;
    const Tst* yj = Y + (int64_t)j * ld;
    double sy = 0.0, yhy = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double y = to_f64(yj[r]);
        sy += to_f64(si[r]) * y;
        const double w = gamma_mode ? y : to_f64(h0[r]) * y;
        yhy += to_f64(yi[r]) * w;
    }
    sy = block_sum<256>(sy, sh);
    yhy = block_sum<256>(yhy, sh);
    if (threadIdx.x == 0) {
        part[((int64_t)i * nbt + b0 + b) * 2 + 0] = sy;
        part[((int64_t)i * nbt + b0 + b) * 2 + 1] = yhy;
    }
}

// Fixed-order sums of the partials; writes column j of Rm and row/column j of YHY.
__global__ void gram_finish_kernel(int j, int kmax, int nb, const double* __restrict__ part,
                                   double* __restrict__ Rm, double* __restrict__ YHY,
                                   double* __restrict__ scalars, int gamma_mode) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > j) return;
    double sy = 0.0, yhy = 0.0;
    for (int b = 0; b < nb; ++b) {
        sy += part[((int64_t)i * nb + b) * 2 + 0];
        yhy += part[((int64_t)i * nb + b) * 2 + 1];
    }
    Rm[(int64_t)j * kmax + i] = sy;
    if (gamma_mode) {
        if (j == 0) scalars[0] = sy / yhy;   // gamma = s_0^T y_0 / y_0^T y_0 (i == j == 0 here)
        yhy *= scalars[0];
    }
    YHY[(int64_t)j * kmax + i] = yhy;
    YHY[(int64_t)i * kmax + j] = yhy;
    if (i == j) {
        scalars[1] = sy;
        scalars[2] = yhy;
    }
}

// Column j of R^-1 for the upper-triangular R = triu(S^T Y), by the column
// recurrence R^-1(0:j, j) = -R^-1(0:j, 0:j) R(0:j, j) / R(j, j).
__global__ void rinv_update_kernel(int j, int kmax, const double* __restrict__ Rm, double* __restrict__ Rinv,
                                   double* __restrict__ RinvT) {
    const double rjj = Rm[(int64_t)j * kmax + j];
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        double v;
        if (i == j) {
            v = 1.0 / rjj;
        } else {
            double s = 0.0;
            for (int l = i; l < j; ++l) s = fma(Rinv[(int64_t)l * kmax + i], Rm[(int64_t)j * kmax + l], s);
            v = -s / rjj;
        }
        Rinv[(int64_t)j * kmax + i] = v;
        RinvT[(int64_t)i * kmax + j] = v;
    }
}

template <typename Th>
__global__ void fill_h0_kernel(int64_t n, Th* __restrict__ h0, const double* __restrict__ scalars) {
    const double g = scalars[0];
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        h0[r] = (Th)g;
}

template <typename Tst, typename To>
__global__ void upcast_kernel(int64_t n, const Tst* __restrict__ src, To* __restrict__ dst) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        dst[r] = (To)to_f64(src[r]);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

template <typename Tin, typename Tst>
static void launch_store(bfgsuq_ctx* h, const void* s, const void* y, int j) {
    Tst* S = (Tst*)h->S + (int64_t)j * h->ld;
    Tst* Y = (Tst*)h->Y + (int64_t)j * h->ld;
    hipLaunchKernelGGL((store_pair_kernel<Tin, Tst>), dim3(grid_for(h->n)), dim3(256), 0, h->stream, h->n,
                       (const Tin*)s, (const Tin*)y, S, Y);
}

template <typename Tst, typename Th>
static void launch_gram(bfgsuq_ctx* h, int j) {
    hipLaunchKernelGGL((gram_partial_kernel<Tst, Th>), dim3(h->gram_blocks, j + 1), dim3(256), 0, h->stream, h->n,
                       h->ld, j, (const Tst*)h->S, (const Tst*)h->Y, (const Th*)h->h0, h->gamma_mode ? 1 : 0,
                       h->gram_part, 0, h->gram_blocks);
}

int stream_slices(bfgsuq_ctx* h, int ncols,
                  const std::function<int(int, int64_t, int64_t, const void*, const void*)>& body) {
    const size_t es = dtype_size(h->storage);
    const int64_t n = h->n, sr = h->slice_rows;
    const int ns = (int)((n + sr - 1) / sr);
    // the copies start after everything already queued on the handle's stream: a push's
    // host write of its column, and the kernels that still read a buffer
    BFGS_HIP(hipEventRecord(h->ev_start, h->stream));
    BFGS_HIP(hipStreamWaitEvent(h->copy_stream, h->ev_start, 0));
    for (int i = 0; i < ns; ++i) {
        const int b = i & 1;
        const int64_t r0 = (int64_t)i * sr, rows = std::min(sr, n - r0);
        if (i >= 2) BFGS_HIP(hipStreamWaitEvent(h->copy_stream, h->ev_free[b], 0));
        for (int w = 0; w < 2; ++w) {
            const char* src = (const char*)(w ? h->Y : h->S) + r0 * es;
            BFGS_HIP(hipMemcpy2DAsync(h->stage[b][w], (size_t)h->slice_ld * es, src, (size_t)h->ld * es, (size_t)rows * es,
                                      (size_t)ncols, hipMemcpyHostToDevice, h->copy_stream));
        }
        BFGS_HIP(hipEventRecord(h->ev_ready[b], h->copy_stream));
        BFGS_HIP(hipStreamWaitEvent(h->stream, h->ev_ready[b], 0));
        const int rc = body(i, r0, rows, h->stage[b][0], h->stage[b][1]);
        if (rc != BFGS_OK) return rc;
        BFGS_HIP(hipEventRecord(h->ev_free[b], h->stream));
    }
    return BFGS_OK;
}

// A streamed history's push: the pair is rounded into device memory, written to its
// host column, and the Gram updates read columns 0 .. j back slice by slice (the same
// O(n j) pass as for a device-resident history, over the host link).
template <typename Tin, typename Tst>
static int store_streamed(bfgsuq_ctx* h, const void* s, const void* y, int j) {
    const size_t es = sizeof(Tst);
    Tst* ts = (Tst*)h->push_tmp;
    Tst* ty = ts + h->n;
    hipLaunchKernelGGL((store_pair_kernel<Tin, Tst>), dim3(grid_for(h->n)), dim3(256), 0, h->stream, h->n,
                       (const Tin*)s, (const Tin*)y, ts, ty);
    BFGS_HIP(hipGetLastError());
    BFGS_HIP(hipMemcpyAsync((char*)h->S + (size_t)j * h->ld * es, ts, (size_t)h->n * es, hipMemcpyDeviceToHost,
                            h->stream));
    BFGS_HIP(hipMemcpyAsync((char*)h->Y + (size_t)j * h->ld * es, ty, (size_t)h->n * es, hipMemcpyDeviceToHost,
                            h->stream));
    return BFGS_OK;
}

template <typename Tst, typename Th>
static int gram_streamed(bfgsuq_ctx* h, int j) {
    const int ns = (int)((h->n + h->slice_rows - 1) / h->slice_rows);
    const int gb = h->gram_blocks / ns;
    return stream_slices(h, j + 1, [&](int i, int64_t r0, int64_t rows, const void* Sst, const void* Yst) {
        hipLaunchKernelGGL((gram_partial_kernel<Tst, Th>), dim3(gb, j + 1), dim3(256), 0, h->stream, rows, h->slice_ld,
                           j, (const Tst*)Sst, (const Tst*)Yst, (const Th*)h->h0 + r0, h->gamma_mode ? 1 : 0,
                           h->gram_part, i * gb, h->gram_blocks);
        return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
    });
}

// push_pair in two halves, so that a batch can enqueue the pushes of many handles
// before it waits for any: push_enqueue stores the pair as column k and queues the
// Gram updates and the copy of (gamma, s^T y, y^T B_0 y) to pinned host memory;
// push_finish waits for the handle's stream and accepts or drops the pair.
int push_enqueue(bfgsuq_ctx* h, const void* s, const void* y, bfgs_dtype in_dtype) {
    if (!h || !s || !y) return BFGS_ERR_ARG;
    if (in_dtype != BFGS_F64 && in_dtype != BFGS_F32) return BFGS_ERR_ARG;
    if (h->k >= h->kmax) return BFGS_ERR_FULL;
    const int j = h->k;
    if (h->streamed) {
        int rc;
        if (h->storage == BFGS_F64) {
            rc = in_dtype == BFGS_F64 ? store_streamed<double, double>(h, s, y, j) : store_streamed<float, double>(h, s, y, j);
            if (rc == BFGS_OK) rc = gram_streamed<double, double>(h, j);
        } else {
            rc = in_dtype == BFGS_F64 ? store_streamed<double, float>(h, s, y, j) : store_streamed<float, float>(h, s, y, j);
            if (rc == BFGS_OK) rc = gram_streamed<float, float>(h, j);
        }
        if (rc != BFGS_OK) return rc;
    } else
    switch (h->storage) {
        case BFGS_F64:
            if (in_dtype == BFGS_F64) launch_store<double, double>(h, s, y, j);
            else launch_store<float, double>(h, s, y, j);
            launch_gram<double, double>(h, j);
            break;
        case BFGS_F32:
            if (in_dtype == BFGS_F64) launch_store<double, float>(h, s, y, j);
            else launch_store<float, float>(h, s, y, j);
            launch_gram<float, float>(h, j);
            break;
        case BFGS_BF16:
            if (in_dtype == BFGS_F64) launch_store<double, bf16_t>(h, s, y, j);
            else launch_store<float, bf16_t>(h, s, y, j);
            if (mfma_scatter_pair(h, j) != BFGS_OK) return BFGS_ERR_HIP;
            launch_gram<bf16_t, float>(h, j);
            break;
    }
    BFGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(gram_finish_kernel, dim3((j + 1 + 255) / 256), dim3(256), 0, h->stream, j, h->kmax,
                       h->gram_blocks, h->gram_part, h->Rm, h->YHY, h->scalars, h->gamma_mode ? 1 : 0);
    BFGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(rinv_update_kernel, dim3(1), dim3(256), 0, h->stream, j, h->kmax, h->Rm, h->Rinv, h->RinvT);
    BFGS_HIP(hipGetLastError());
    BFGS_HIP(hipMemcpyAsync(h->host_sc, h->scalars, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return BFGS_OK;
}

int push_finish(bfgsuq_ctx* h) {
    const int j = h->k;
    BFGS_HIP(hipStreamSynchronize(h->stream));
    const double g = h->host_sc[0], sy = h->host_sc[1], yhy = h->host_sc[2];
    if (!std::isfinite(sy) || !std::isfinite(yhy) || (h->gamma_mode && j == 0 && !std::isfinite(g)))
        return BFGS_ERR_NONFINITE;
    if (!(sy > 0.0)) return BFGS_ERR_CURVATURE;
    if (h->gamma_mode && j == 0) {
        if (!(g > 0.0)) return BFGS_ERR_CURVATURE;
        if (h->storage == BFGS_F64)
            hipLaunchKernelGGL(fill_h0_kernel<double>, dim3(grid_for(h->n)), dim3(256), 0, h->stream, h->n,
                               (double*)h->h0, (const double*)h->scalars);
        else
            hipLaunchKernelGGL(fill_h0_kernel<float>, dim3(grid_for(h->n)), dim3(256), 0, h->stream, h->n,
                               (float*)h->h0, (const double*)h->scalars);
        BFGS_HIP(hipGetLastError());
        h->gamma_known = true;
    }
    h->k = j + 1;
    ++h->gen;
    h->have_rsvd = false;
    return BFGS_OK;
}

// Forgetting the oldest pair (the limited-memory form): column j of S and Y moves to
// column j - 1 for j = 1 .. k-1.  A thread moves one row of both, in increasing j, so
// every value is read before its slot is overwritten.
template <typename T>
__global__ void shift_pairs_kernel(int64_t n, int64_t ld, int k, T* __restrict__ S, T* __restrict__ Y) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        for (int j = 1; j < k; ++j) {
            S[(int64_t)(j - 1) * ld + r] = S[(int64_t)j * ld + r];
            Y[(int64_t)(j - 1) * ld + r] = Y[(int64_t)j * ld + r];
        }
    }
}

// The small matrices lose their first row and column: entry (i + 1, j + 1) moves to
// (i, j).  One thread per diagonal d = j - i walks it in increasing i, so every entry
// is read before it is overwritten.  The inverse of R's trailing block is the trailing
// block of R^-1 (R is upper triangular), so R^-1 and its transpose shift like R.
__global__ void shift_small_kernel(int k, int kmax, double* __restrict__ Rm, double* __restrict__ YHY,
                                   double* __restrict__ Rinv, double* __restrict__ RinvT) {
    const int d = (int)(blockIdx.x * blockDim.x + threadIdx.x) - (k - 2);   // -(k-2) .. k-2
    if (d > k - 2) return;
    for (int i = d < 0 ? -d : 0; i < k - 1 && i + d < k - 1; ++i) {
        const int64_t to = (int64_t)(i + d) * kmax + i, from = (int64_t)(i + d + 1) * kmax + (i + 1);
        Rm[to] = Rm[from];
        YHY[to] = YHY[from];
        Rinv[to] = Rinv[from];
        RinvT[to] = RinvT[from];
    }
}

int pop_oldest(bfgsuq_ctx* h) {
    if (h->storage == BFGS_BF16) return BFGS_ERR_ARG;   // its matrix-core layouts group the pairs by 16
    if (h->streamed) return BFGS_ERR_STATE;
    if (h->k < 1) return BFGS_ERR_STATE;
    const int k = h->k;
    if (k > 1) {
        if (h->storage == BFGS_F64)
            hipLaunchKernelGGL(shift_pairs_kernel<double>, dim3(grid_for(h->n)), dim3(256), 0, h->stream, h->n, h->ld,
                               k, (double*)h->S, (double*)h->Y);
        else
            hipLaunchKernelGGL(shift_pairs_kernel<float>, dim3(grid_for(h->n)), dim3(256), 0, h->stream, h->n, h->ld,
                               k, (float*)h->S, (float*)h->Y);
        BFGS_HIP(hipGetLastError());
        hipLaunchKernelGGL(shift_small_kernel, dim3((2 * k - 3 + 63) / 64), dim3(64), 0, h->stream, k, h->kmax, h->Rm,
                           h->YHY, h->Rinv, h->RinvT);
        BFGS_HIP(hipGetLastError());
    }
    h->k = k - 1;
    ++h->gen;
    h->have_rsvd = false;
    return BFGS_OK;
}

extern "C" {

int bfgs_pop_oldest(bfgs_t h) {
    if (!h) return BFGS_ERR_ARG;
    return pop_oldest(h);
}

const char* bfgs_status_string(int code) {
    switch (code) {
        case BFGS_OK: return "ok";
        case BFGS_ERR_ARG: return "invalid argument";
        case BFGS_ERR_FULL: return "pair storage full";
        case BFGS_ERR_STATE: return "call out of order";
        case BFGS_ERR_CURVATURE: return "stored pair has s^T y <= 0";
        case BFGS_ERR_NONFINITE: return "non-finite value";
        case BFGS_ERR_NUMERIC: return "numerical breakdown";
        case BFGS_ERR_ALLOC: return "device allocation failed";
        case BFGS_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

int bfgs_destroy(bfgs_t h) {
    if (!h) return BFGS_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->copy_stream) (void)hipStreamSynchronize(h->copy_stream);
    if (h->streamed) {
        if (h->S) (void)hipHostFree(h->S);
        if (h->Y) (void)hipHostFree(h->Y);
        h->S = h->Y = nullptr;
        void* st[] = {h->stage[0][0], h->stage[0][1], h->stage[1][0], h->stage[1][1], h->push_tmp};
        for (void* p : st)
            if (p) (void)hipFree(p);
        hipEvent_t evs[] = {h->ev_ready[0], h->ev_ready[1], h->ev_free[0], h->ev_free[1], h->ev_start};
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
        if (h->copy_stream) (void)hipStreamDestroy(h->copy_stream);
    }
    void* ptrs[] = {h->S, h->Y, h->h0, h->Rm, h->YHY, h->Rinv, h->RinvT, h->gram_part, h->scalars, h->status,
                    h->S1, h->Y1, h->S2, h->Y2};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    Workspace* ws[] = {&h->part, &h->Z, &h->PT, &h->small16, &h->X, &h->E, &h->Q, &h->W, &h->refl, &h->tau,
                       &h->Rtree, &h->small, &h->lam, &h->diag};
    for (Workspace* w : ws) free_ws(*w);
    for (hipEvent_t e : h->prof.pool) (void)hipEventDestroy(e);
    if (h->host_sc) (void)hipHostFree(h->host_sc);
    delete h;
    return BFGS_OK;
}

}  // extern "C"

// slice_rows = 0: S and Y in device memory; > 0: in pinned host memory, streamed.
static int create_impl(int64_t n, int32_t k_max, const void* H0, bfgs_dtype storage, void* stream,
                       int64_t slice_rows, bfgs_t* out) {
    if (!out) return BFGS_ERR_ARG;
    *out = nullptr;
    if (n < 1 || k_max < 1 || k_max > BFGS_MAX_PAIRS || slice_rows < 0) return BFGS_ERR_ARG;
    if (storage != BFGS_F64 && storage != BFGS_F32 && storage != BFGS_BF16) return BFGS_ERR_ARG;
    if (slice_rows > 0 && storage == BFGS_BF16) return BFGS_ERR_ARG;
    bfgsuq_ctx* h = new (std::nothrow) bfgsuq_ctx();
    if (!h) return BFGS_ERR_ALLOC;
    h->n = n;
    h->ld = round_up(n, 128);
    h->kmax = k_max;
    h->storage = storage;
    h->stream = (hipStream_t)stream;
    h->gamma_mode = (H0 == nullptr);
    const size_t es = dtype_size(storage);
    const size_t hs = storage == BFGS_F64 ? 8 : 4;
    h->gram_blocks = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 4095) / 4096));
    if (slice_rows > 0) {
        h->streamed = true;
        h->slice_rows = std::min(slice_rows, n);
        h->slice_ld = round_up(h->slice_rows, 128);
        // per slice the Gram partials of a push: gram_blocks = slices x per-slice blocks
        const int64_t ns = (n + h->slice_rows - 1) / h->slice_rows;
        const int64_t gb = std::min<int64_t>(64, std::max<int64_t>(1, (h->slice_rows + 4095) / 4096));
        if (ns * gb > (1 << 20)) {
            delete h;
            return BFGS_ERR_ARG;
        }
        h->gram_blocks = (int)(ns * gb);
    }
    int rc = BFGS_OK;
    auto alloc = [&](void** p, size_t bytes) {
        if (rc != BFGS_OK) return;
        if (hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            rc = BFGS_ERR_ALLOC;
        }
    };
    const size_t hist_bytes = (size_t)h->ld * k_max * es;
    if (h->streamed) {
        auto halloc = [&](void** p) {
            if (rc != BFGS_OK) return;
            if (hipHostMalloc(p, hist_bytes, hipHostMallocDefault) != hipSuccess) {
                *p = nullptr;
                rc = BFGS_ERR_ALLOC;
                return;
            }
            std::memset(*p, 0, hist_bytes);
        };
        halloc(&h->S);
        halloc(&h->Y);
        for (int b = 0; b < 2; ++b)
            for (int w = 0; w < 2; ++w) alloc(&h->stage[b][w], (size_t)h->slice_ld * k_max * es);
        alloc(&h->push_tmp, 2 * (size_t)n * es);
        if (rc == BFGS_OK && hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking) != hipSuccess) {
            h->copy_stream = nullptr;
            rc = BFGS_ERR_HIP;
        }
        hipEvent_t* evs[] = {&h->ev_ready[0], &h->ev_ready[1], &h->ev_free[0], &h->ev_free[1], &h->ev_start};
        for (hipEvent_t* e : evs)
            if (rc == BFGS_OK && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
                *e = nullptr;
                rc = BFGS_ERR_HIP;
            }
    } else {
        alloc(&h->S, hist_bytes);
        alloc(&h->Y, hist_bytes);
    }
    alloc(&h->h0, (size_t)h->ld * hs);
    alloc((void**)&h->Rm, (size_t)k_max * k_max * 8);
    alloc((void**)&h->YHY, (size_t)k_max * k_max * 8);
    alloc((void**)&h->Rinv, (size_t)k_max * k_max * 8);
    alloc((void**)&h->RinvT, (size_t)k_max * k_max * 8);
    alloc((void**)&h->gram_part, (size_t)k_max * h->gram_blocks * 2 * 8);
    alloc((void**)&h->scalars, 8 * 8);
    alloc((void**)&h->status, 64);
    if (rc == BFGS_OK && hipHostMalloc((void**)&h->host_sc, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        h->host_sc = nullptr;
        rc = BFGS_ERR_ALLOC;
    }
    size_t f1_bytes = 0, f2_bytes = 0;
    if (storage == BFGS_BF16) {
        f1_bytes = (size_t)mfma_rows_f1(n) * k_max * 2;
        f2_bytes = (size_t)mfma_rows_f2(n) * mfma_groups(k_max) * 16 * 2;
        alloc(&h->S1, f1_bytes);
        alloc(&h->Y1, f1_bytes);
        alloc(&h->S2, f2_bytes);
        alloc(&h->Y2, f2_bytes);
    }
    if (rc != BFGS_OK) {
        bfgs_destroy(h);
        return rc;
    }
    if ((!h->streamed && (hipMemsetAsync(h->S, 0, hist_bytes, h->stream) != hipSuccess ||
                          hipMemsetAsync(h->Y, 0, hist_bytes, h->stream) != hipSuccess)) ||
        hipMemsetAsync(h->h0, 0, (size_t)h->ld * hs, h->stream) != hipSuccess ||
        hipMemsetAsync(h->Rm, 0, (size_t)k_max * k_max * 8, h->stream) != hipSuccess ||
        hipMemsetAsync(h->YHY, 0, (size_t)k_max * k_max * 8, h->stream) != hipSuccess ||
        hipMemsetAsync(h->Rinv, 0, (size_t)k_max * k_max * 8, h->stream) != hipSuccess ||
        hipMemsetAsync(h->RinvT, 0, (size_t)k_max * k_max * 8, h->stream) != hipSuccess ||
        hipMemsetAsync(h->scalars, 0, 64, h->stream) != hipSuccess ||
        hipMemsetAsync(h->status, 0, 64, h->stream) != hipSuccess ||
        (f1_bytes && (hipMemsetAsync(h->S1, 0, f1_bytes, h->stream) != hipSuccess ||
                      hipMemsetAsync(h->Y1, 0, f1_bytes, h->stream) != hipSuccess ||
                      hipMemsetAsync(h->S2, 0, f2_bytes, h->stream) != hipSuccess ||
                      hipMemsetAsync(h->Y2, 0, f2_bytes, h->stream) != hipSuccess))) {
        bfgs_destroy(h);
        return BFGS_ERR_HIP;
    }
    if (H0) {
        if (hipMemcpyAsync(h->h0, H0, (size_t)n * hs, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) {
            bfgs_destroy(h);
            return BFGS_ERR_HIP;
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        bfgs_destroy(h);
        return BFGS_ERR_HIP;
    }
    *out = h;
    return BFGS_OK;
}

extern "C" {

int bfgs_create(int64_t n, int32_t k_max, const void* H0, bfgs_dtype storage, void* stream, bfgs_t* out) {
    return create_impl(n, k_max, H0, storage, stream, 0, out);
}

int bfgs_create_streamed(int64_t n, int32_t k_max, const void* H0, bfgs_dtype storage, int64_t slice_rows,
                         void* stream, bfgs_t* out) {
    if (slice_rows < 1) return BFGS_ERR_ARG;
    return create_impl(n, k_max, H0, storage, stream, slice_rows, out);
}

int bfgs_num_pairs(bfgs_t h, int32_t* k_out) {
    if (!h || !k_out) return BFGS_ERR_ARG;
    *k_out = h->k;
    return BFGS_OK;
}

int bfgs_push_pair(bfgs_t h, const void* s, const void* y, bfgs_dtype in_dtype) {
    const int rc = push_enqueue(h, s, y, in_dtype);
    return rc != BFGS_OK ? rc : push_finish(h);
}

int bfgs_apply_Hinv(bfgs_t h, const void* V, int32_t ncols, void* out) {
    if (!h || !V || !out || ncols < 1 || ncols > BFGS_MAX_COLS) return BFGS_ERR_ARG;
    if (V == out) return BFGS_ERR_ARG;
    if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    return apply_block(h, V, ncols, out, false);
}

int bfgs_apply_Hdiff(bfgs_t h, const void* V, int32_t ncols, void* out) {
    if (!h || !V || !out || ncols < 1 || ncols > BFGS_MAX_COLS) return BFGS_ERR_ARG;
    if (V == out) return BFGS_ERR_ARG;
    if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    return apply_block(h, V, ncols, out, true);
}

int bfgs_get_pair(bfgs_t h, int32_t j, void* s_out, void* y_out) {
    if (!h || j < 0 || j >= h->k) return BFGS_ERR_ARG;
    const int64_t off = (int64_t)j * h->ld;
    for (int w = 0; w < 2; ++w) {
        void* dst = w == 0 ? s_out : y_out;
        if (!dst) continue;
        const void* base = w == 0 ? h->S : h->Y;
        switch (h->storage) {
            case BFGS_F64:
                hipLaunchKernelGGL((upcast_kernel<double, double>), dim3(grid_for(h->n)), dim3(256), 0, h->stream,
                                   h->n, (const double*)base + off, (double*)dst);
                break;
            case BFGS_F32:
                hipLaunchKernelGGL((upcast_kernel<float, float>), dim3(grid_for(h->n)), dim3(256), 0, h->stream,
                                   h->n, (const float*)base + off, (float*)dst);
                break;
            case BFGS_BF16:
                hipLaunchKernelGGL((upcast_kernel<bf16_t, float>), dim3(grid_for(h->n)), dim3(256), 0, h->stream,
                                   h->n, (const bf16_t*)base + off, (float*)dst);
                break;
        }
        BFGS_HIP(hipGetLastError());
    }
    return BFGS_OK;
}

int bfgs_get_h0(bfgs_t h, void* out) {
    if (!h || !out) return BFGS_ERR_ARG;
    if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    const size_t hs = h->storage == BFGS_F64 ? 8 : 4;
    BFGS_HIP(hipMemcpyAsync(out, h->h0, (size_t)h->n * hs, hipMemcpyDeviceToDevice, h->stream));
    return BFGS_OK;
}

int bfgs_get_status(bfgs_t h) {
    if (!h) return BFGS_ERR_ARG;
    int32_t st = 0;
    BFGS_HIP(hipMemcpyAsync(&st, h->status, 4, hipMemcpyDeviceToHost, h->stream));
    BFGS_HIP(hipStreamSynchronize(h->stream));
    if (st != 0) {
        BFGS_HIP(hipMemsetAsync(h->status, 0, 4, h->stream));
        BFGS_HIP(hipStreamSynchronize(h->stream));
    }
    return st;
}

int bfgs_generate_probes(bfgs_t h, uint64_t seed, int32_t ncols, void* X) {
    if (!h || !X || ncols < 1 || ncols > BFGS_MAX_COLS) return BFGS_ERR_ARG;
    return probes_run(h, seed, ncols, X);
}

int bfgs_rsvd(bfgs_t h, int32_t rank, int32_t oversample, uint64_t seed, void* U, double* Sigma) {
    if (!h || !U || !Sigma || rank < 1 || oversample < 0) return BFGS_ERR_ARG;
    const int64_t c = (int64_t)rank + oversample;
    if (c > BFGS_MAX_COLS || c > h->n) return BFGS_ERR_ARG;
    if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    return rsvd_run(h, rank, oversample, seed, U, Sigma);
}

int bfgs_rsvd_ex(bfgs_t h, int32_t rank, int32_t oversample, uint64_t seed, uint32_t flags, void* U, double* Sigma) {
    if (!h || !U || !Sigma || rank < 1 || oversample < 0) return BFGS_ERR_ARG;
    if (flags & ~(BFGS_RSVD_PRECOND | BFGS_RSVD_TWO_PASS)) return BFGS_ERR_ARG;
    const int64_t c = (int64_t)rank + oversample;
    if (c > BFGS_MAX_COLS || c > h->n) return BFGS_ERR_ARG;
    if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    return rsvd_run(h, rank, oversample, seed, U, Sigma, flags);
}

int bfgs_profile(bfgs_t h, int32_t enable) {
    if (!h) return BFGS_ERR_ARG;
    h->prof.on = enable != 0;
    return BFGS_OK;
}

int bfgs_profile_report(bfgs_t h, char* buf, int32_t len) {
    if (!h || !buf || len < 3) return BFGS_ERR_ARG;
    BFGS_HIP(hipStreamSynchronize(h->stream));
    std::vector<const char*> names;
    std::vector<double> tot;
    std::vector<int> cnt;
    for (const ProfRec& r : h->prof.recs) {
        float ms = 0.f;
        if (!r.ended) continue;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            (void)hipGetLastError();   // leave no error behind for the caller's next HIP call
            continue;
        }
        size_t i = 0;
        for (; i < names.size(); ++i)
            if (std::strcmp(names[i], r.name) == 0) break;
        if (i == names.size()) {
            names.push_back(r.name);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[i] += ms;
        cnt[i] += 1;
    }
    h->prof.recs.clear();
    h->prof.open.clear();
    h->prof.used = 0;
    int off = std::snprintf(buf, len, "{");
    for (size_t i = 0; i < names.size() && off < len; ++i)
        off += std::snprintf(buf + off, len - off, "%s\"%s\": [%d, %.6f]", i ? ", " : "", names[i], cnt[i], tot[i]);
    if (off < len) std::snprintf(buf + off, len - off, "}");
    return off < len - 1 ? BFGS_OK : BFGS_ERR_ARG;
}

int bfgs_posterior_diag(bfgs_t h, void* out) {
    if (!h || !out) return BFGS_ERR_ARG;
    if (!h->have_rsvd) return BFGS_ERR_STATE;
    const size_t hs = h->storage == BFGS_F64 ? 8 : 4;
    BFGS_HIP(hipMemcpyAsync(out, h->diag.ptr, (size_t)h->n * hs, hipMemcpyDeviceToDevice, h->stream));
    return BFGS_OK;
}

}  // extern "C"
