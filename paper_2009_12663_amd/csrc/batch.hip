// Batched form: many independent inversions (uneven n and k) driven together.
//
// A batch owns one handle per problem.  With float32 or float64 storage (and
// 1 <= k <= 256 everywhere) the apply of all problems is four launches in all:
// persistent pass kernels take (problem, tile) items from a work queue, longest
// problems first (batch_apply_persistent).  Otherwise, and for the rSVD, problems
// are spread over a small set of side streams forked from the caller's stream with
// events and joined back, so their kernels overlap on the device.  Apply + rSVD of
// every problem can be captured once into a hipGraph and replayed with a single
// launch.  The autotuner times the tunable launch shapes of each problem (rows per
// pass-1 workgroup, TSQR chain count) and the persistent grid (workgroups per
// compute unit) with HIP events and keeps the fastest.
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

struct bfgsuq_batch {
    int nprob = 0;
    hipStream_t main = nullptr;
    hipStream_t cap = nullptr;            // graph capture / replay stream (the caller's may be the null stream)
    hipEvent_t cap_in = nullptr, cap_out = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    std::vector<bfgsuq_ctx*> h;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // handle_generation() of every problem when the graph was captured: the graph holds
    // each handle's k, tunables and workspace pointers, so any later change invalidates it
    std::vector<unsigned long long> captured_gen;
    // persistent apply: descriptors for eager calls [0] and for the captured graph [1]
    PersistSlot pslot[2];
    int wg_per_cu = 2;
};

namespace {

constexpr int MAX_SIDE_STREAMS = 8;

template <typename F>
int forked(bfgsuq_batch* b, hipStream_t root, F&& fn) {
    BFGS_HIP(hipEventRecord(b->fork, root));
    for (hipStream_t s : b->side) BFGS_HIP(hipStreamWaitEvent(s, b->fork, 0));
    int first = BFGS_OK;
    for (int i = 0; i < b->nprob; ++i) {
        const int rc = fn(i);
        if (rc != BFGS_OK && first == BFGS_OK) first = rc;
    }
    for (size_t s = 0; s < b->side.size(); ++s) {
        BFGS_HIP(hipEventRecord(b->join[s], b->side[s]));
        BFGS_HIP(hipStreamWaitEvent(root, b->join[s], 0));
    }
    return first;
}

// Every side stream's work so far ordered before fn's work on root, and fn's work
// before anything queued on the side streams afterwards.
template <typename F>
int joined(bfgsuq_batch* b, hipStream_t root, F&& fn) {
    for (size_t s = 0; s < b->side.size(); ++s) {
        BFGS_HIP(hipEventRecord(b->join[s], b->side[s]));
        BFGS_HIP(hipStreamWaitEvent(root, b->join[s], 0));
    }
    const int rc = fn();
    BFGS_HIP(hipEventRecord(b->fork, root));
    for (hipStream_t s : b->side) BFGS_HIP(hipStreamWaitEvent(s, b->fork, 0));
    return rc;
}

bool persistent_ok(const bfgsuq_batch* b) {
    const bfgs_dtype s0 = b->h[0]->storage;
    if (s0 != BFGS_F32 && s0 != BFGS_F64) return false;
    for (const bfgsuq_ctx* h : b->h)
        if (h->storage != s0 || h->streamed || h->k < 1 || h->k > 256) return false;
    return true;
}

// capture: root is capturing and the apply opens the captured work, so it needs no
// join (events recorded outside a capture cannot be waited for inside it); the rSVD
// forked after it orders the side streams behind it.
int batch_apply(bfgsuq_batch* b, hipStream_t root, const void* const* V, const int32_t* ncols, void* const* out,
                int slot, bool upload, bool capture = false) {
    if (persistent_ok(b)) {
        auto launch = [&] {
            return batch_apply_persistent(b->h.data(), b->nprob, V, ncols, out, root, &b->pslot[slot], upload,
                                          b->wg_per_cu);
        };
        return capture ? launch() : joined(b, root, launch);
    }
    return forked(b, root, [&](int i) { return apply_block(b->h[i], V[i], ncols[i], out[i], false); });
}

void destroy_graph(bfgsuq_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured_gen.clear();
}

// Mean time (ms) of `reps` calls of fn on the handle's stream.
template <typename F>
float time_ms(bfgsuq_ctx* h, int reps, F&& fn) {
    hipEvent_t a, z;
    if (hipEventCreate(&a) != hipSuccess) return 1e30f;
    if (hipEventCreate(&z) != hipSuccess) {
        (void)hipEventDestroy(a);
        return 1e30f;
    }
    fn();   // warm (allocations, attributes)
    (void)hipEventRecord(a, h->stream);
    for (int r = 0; r < reps; ++r) fn();
    (void)hipEventRecord(z, h->stream);
    (void)hipEventSynchronize(z);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, z);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    return ms / reps;
}

}  // namespace

extern "C" {

int bfgs_autotune(bfgs_t h, int32_t ncols, int32_t rank, int32_t oversample, void* V, void* out, void* U,
                  double* Sigma) {
    if (!h || !V || !out || ncols < 1 || ncols > BFGS_MAX_COLS || h->k < 1) return BFGS_ERR_ARG;
    if (mfma_apply_supported(h, ncols)) {
        const int cand[] = {64, 128, 256, 512};
        float best = 1e30f;
        int best_nk = h->g1_nk;
        for (int nk : cand) {
            h->g1_nk = nk;
            const float t = time_ms(h, 3, [&] { (void)apply_block(h, V, ncols, out, false); });
            if (t < best) {
                best = t;
                best_nk = nk;
            }
        }
        h->g1_nk = best_nk;
    }
    if (U && Sigma && rank >= 1 && oversample >= 0 && rank + oversample <= ncols) {
        const int cand[] = {64, 128, 256};
        float best = 1e30f;
        int best_ch = h->qr_chains;
        for (int ch : cand) {
            h->qr_chains = ch;
            const float t = time_ms(h, 1, [&] { (void)rsvd_run(h, rank, oversample, 1, U, Sigma); });
            if (t < best) {
                best = t;
                best_ch = ch;
            }
        }
        h->qr_chains = best_ch;
    }
    ++h->gen;   // launch shapes may have changed
    return hipStreamSynchronize(h->stream) == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int bfgs_sync(bfgs_t h) {
    if (!h) return BFGS_ERR_ARG;
    return hipStreamSynchronize(h->stream) == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int bfgs_tuning(bfgs_t h, int32_t* g1_rows, int32_t* qr_chains) {
    if (!h) return BFGS_ERR_ARG;
    if (g1_rows) *g1_rows = h->g1_nk;
    if (qr_chains) *qr_chains = h->qr_chains;
    return BFGS_OK;
}

int bfgs_set_tuning(bfgs_t h, int32_t g1_rows, int32_t qr_chains) {
    if (!h) return BFGS_ERR_ARG;
    // the TSQR tree pairs chains: a power of two, at most the partials' 256
    const bool g1_ok = g1_rows <= 0 || (g1_rows >= 8 && g1_rows <= 1024);
    const bool qr_ok = qr_chains <= 0 || (qr_chains <= 256 && (qr_chains & (qr_chains - 1)) == 0);
    if (!g1_ok || !qr_ok) return BFGS_ERR_ARG;
    if (g1_rows > 0) h->g1_nk = g1_rows;
    if (qr_chains > 0) h->qr_chains = qr_chains;
    ++h->gen;   // launch shapes may have changed
    return BFGS_OK;
}

int bfgs_batch_destroy(bfgs_batch_t b) {
    if (!b) return BFGS_OK;
    (void)hipStreamSynchronize(b->main);
    destroy_graph(b);
    for (bfgsuq_ctx* h : b->h) bfgs_destroy(h);
    for (PersistSlot& ps : b->pslot) {
        if (ps.prob) (void)hipFree(ps.prob);
        if (ps.head) (void)hipFree(ps.head);
    }
    for (hipStream_t s : b->side) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap) {
        (void)hipStreamSynchronize(b->cap);
        (void)hipStreamDestroy(b->cap);
    }
    if (b->cap_in) (void)hipEventDestroy(b->cap_in);
    if (b->cap_out) (void)hipEventDestroy(b->cap_out);
    delete b;
    return BFGS_OK;
}

int bfgs_batch_create(int32_t nprob, const int64_t* n, const int32_t* k_max, const void* const* H0, bfgs_dtype storage,
                      void* stream, bfgs_batch_t* out) {
    if (!out || !n || !k_max || nprob < 1) return BFGS_ERR_ARG;
    *out = nullptr;
    bfgsuq_batch* b = new (std::nothrow) bfgsuq_batch();
    if (!b) return BFGS_ERR_ALLOC;
    b->nprob = nprob;
    b->main = (hipStream_t)stream;
    const int ns = nprob < MAX_SIDE_STREAMS ? nprob : MAX_SIDE_STREAMS;
    int rc = BFGS_OK;
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->cap_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->cap_out, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        rc = BFGS_ERR_HIP;
    for (int s = 0; s < ns && rc == BFGS_OK; ++s) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            rc = BFGS_ERR_HIP;
            break;
        }
        b->side.push_back(st);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            rc = BFGS_ERR_HIP;
            break;
        }
        b->join.push_back(ev);
    }
    for (int i = 0; i < nprob && rc == BFGS_OK; ++i) {
        bfgs_t h = nullptr;
        rc = bfgs_create(n[i], k_max[i], H0 ? H0[i] : nullptr, storage, b->side[i % ns], &h);
        if (rc == BFGS_OK) b->h.push_back(h);
    }
    if (rc != BFGS_OK) {
        bfgs_batch_destroy(b);
        return rc;
    }
    *out = b;
    return BFGS_OK;
}

int bfgs_batch_handle(bfgs_batch_t b, int32_t i, bfgs_t* h_out) {
    if (!b || !h_out || i < 0 || i >= b->nprob) return BFGS_ERR_ARG;
    *h_out = b->h[i];
    return BFGS_OK;
}

int bfgs_batch_push_pairs(bfgs_batch_t b, const void* const* S, const void* const* Y, const int32_t* kcount,
                          bfgs_dtype in_dtype) {
    if (!b || !S || !Y || !kcount) return BFGS_ERR_ARG;
    if (in_dtype != BFGS_F64 && in_dtype != BFGS_F32) return BFGS_ERR_ARG;
    int kmax = 0;
    for (int i = 0; i < b->nprob; ++i) {
        if (kcount[i] < 0 || (kcount[i] > 0 && (!S[i] || !Y[i]))) return BFGS_ERR_ARG;
        if (b->h[i]->k + kcount[i] > b->h[i]->kmax) return BFGS_ERR_FULL;
        kmax = kcount[i] > kmax ? kcount[i] : kmax;
    }
    const size_t es = in_dtype == BFGS_F64 ? 8 : 4;
    int first = BFGS_OK;
    // round j: pair j of every problem is queued on the problem's stream, then each
    // problem's check waits for its own stream only, so the pushes of the problems overlap
    for (int j = 0; j < kmax; ++j) {
        std::vector<int> queued(b->nprob, 0);
        for (int i = 0; i < b->nprob; ++i) {
            if (j >= kcount[i]) continue;
            bfgsuq_ctx* h = b->h[i];
            const size_t off = (size_t)j * (size_t)h->n * es;
            const int rc = push_enqueue(h, (const char*)S[i] + off, (const char*)Y[i] + off, in_dtype);
            if (rc != BFGS_OK) {
                if (first == BFGS_OK) first = rc;
            } else {
                queued[i] = 1;
            }
        }
        for (int i = 0; i < b->nprob; ++i) {
            if (!queued[i]) continue;
            const int rc = push_finish(b->h[i]);
            if (rc != BFGS_OK && first == BFGS_OK) first = rc;
        }
    }
    return first;
}

int bfgs_batch_apply_Hinv(bfgs_batch_t b, const void* const* V, const int32_t* ncols, void* const* out) {
    if (!b || !V || !ncols || !out) return BFGS_ERR_ARG;
    for (int i = 0; i < b->nprob; ++i)
        if (!V[i] || !out[i] || ncols[i] < 1 || ncols[i] > BFGS_MAX_COLS || V[i] == out[i] ||
            (b->h[i]->gamma_mode && !b->h[i]->gamma_known))
            return BFGS_ERR_ARG;
    return batch_apply(b, b->main, V, ncols, out, 0, true);
}

int bfgs_batch_rsvd(bfgs_batch_t b, const int32_t* rank, int32_t oversample, uint64_t seed, void* const* U,
                    double* const* Sigma) {
    if (!b || !rank || !U || !Sigma || oversample < 0) return BFGS_ERR_ARG;
    for (int i = 0; i < b->nprob; ++i) {
        bfgsuq_ctx* h = b->h[i];
        const int64_t c = (int64_t)rank[i] + oversample;
        if (rank[i] < 1 || c > BFGS_MAX_COLS || c > h->n || !U[i] || !Sigma[i]) return BFGS_ERR_ARG;
        if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    }
    return forked(b, b->main, [&](int i) { return rsvd_run(b->h[i], rank[i], oversample, seed + (uint64_t)i, U[i], Sigma[i]); });
}

int bfgs_batch_autotune(bfgs_batch_t b, const void* const* V, const int32_t* ncols, void* const* out,
                        const int32_t* rank, int32_t oversample, void* const* U, double* const* Sigma) {
    if (!b || !V || !ncols || !out) return BFGS_ERR_ARG;
    for (int i = 0; i < b->nprob; ++i) {
        const int rc = bfgs_autotune(b->h[i], ncols[i], rank ? rank[i] : 0, oversample, (void*)V[i], out[i],
                                     U ? U[i] : nullptr, Sigma ? Sigma[i] : nullptr);
        if (rc != BFGS_OK) return rc;
    }
    if (persistent_ok(b)) {
        // the persistent grid: workgroups per compute unit
        const int cand[] = {1, 2, 4};
        float best = 1e30f;
        int best_w = b->wg_per_cu;
        hipEvent_t e0, e1;
        BFGS_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return BFGS_ERR_HIP;
        }
        int rc = BFGS_OK;
        for (int w : cand) {
            b->wg_per_cu = w;
            rc = batch_apply(b, b->main, V, ncols, out, 0, true);   // warm, uploads the descriptors
            if (rc != BFGS_OK) break;
            (void)hipEventRecord(e0, b->main);
            for (int r = 0; r < 3 && rc == BFGS_OK; ++r) rc = batch_apply(b, b->main, V, ncols, out, 0, false);
            (void)hipEventRecord(e1, b->main);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rc == BFGS_OK && ms < best) {
                best = ms;
                best_w = w;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->wg_per_cu = best_w;
        for (bfgsuq_ctx* h : b->h) ++h->gen;   // the persistent grid is part of a captured graph
        if (rc != BFGS_OK) return rc;
    }
    return BFGS_OK;
}

int bfgs_batch_graph_build(bfgs_batch_t b, const void* const* V, const int32_t* ncols, void* const* out,
                           const int32_t* rank, int32_t oversample, uint64_t seed, void* const* U,
                           double* const* Sigma) {
    if (!b) return BFGS_ERR_ARG;
    // One eager pass sizes every workspace (and fills the graph's persistent
    // descriptors), so nothing is allocated or copied while capturing.
    int rc = bfgs_batch_apply_Hinv(b, V, ncols, out);
    if (rc == BFGS_OK && persistent_ok(b)) rc = batch_apply(b, b->main, V, ncols, out, 1, true);
    if (rc == BFGS_OK) rc = bfgs_batch_rsvd(b, rank, oversample, seed, U, Sigma);
    if (rc != BFGS_OK) return rc;
    BFGS_HIP(hipStreamSynchronize(b->main));
    destroy_graph(b);
    BFGS_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    rc = batch_apply(b, b->cap, V, ncols, out, 1, false, true);
    if (rc == BFGS_OK)
        rc = forked(b, b->cap, [&](int i) {
            return rsvd_run(b->h[i], rank[i], oversample, seed + (uint64_t)i, U[i], Sigma[i]);
        });
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != BFGS_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != BFGS_OK ? rc : BFGS_ERR_HIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        destroy_graph(b);
        return BFGS_ERR_HIP;
    }
    for (bfgsuq_ctx* h : b->h) b->captured_gen.push_back(handle_generation(h));
    return BFGS_OK;
}

int bfgs_batch_graph_launch(bfgs_batch_t b) {
    if (!b) return BFGS_ERR_ARG;
    if (!b->exec) return BFGS_ERR_STATE;
    for (int i = 0; i < b->nprob; ++i)
        if (handle_generation(b->h[i]) != b->captured_gen[i]) {
            // a push, a retune or a workspace reallocation since the capture: the graph
            // would replay stale sizes or freed buffers
            destroy_graph(b);
            return BFGS_ERR_STATE;
        }
    BFGS_HIP(hipEventRecord(b->cap_in, b->main));
    BFGS_HIP(hipStreamWaitEvent(b->cap, b->cap_in, 0));
    BFGS_HIP(hipGraphLaunch(b->exec, b->cap));
    BFGS_HIP(hipEventRecord(b->cap_out, b->cap));
    BFGS_HIP(hipStreamWaitEvent(b->main, b->cap_out, 0));
    return BFGS_OK;
}

}  // extern "C"
