// bfgs_apply_Hinv without device allocation, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The apply's scratch (split-K partials of pass 1, Z, P, T and the bfloat16 small
// operand of pass 2) comes from one file-scope device array instead of the
// handle's grow-only workspaces.  Every GPU holds its own copy of the array for
// the life of the process; its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to kernels.  All calls on one GPU share the array: calls that overlap on
// one GPU (different streams, or different handles without ordering) race.  The
// apply kernels write every scratch element they later read, so nothing has to
// be cleared between calls.
#include <mutex>

#include "common.h"

namespace {

constexpr size_t kZBytes = (size_t)2 * BFGS_MAX_PAIRS * BFGS_MAX_COLS * sizeof(double);   // 4 MiB
constexpr size_t kPTBytes = kZBytes;                                                      // 4 MiB
constexpr size_t kSmall16Bytes = (size_t)2 * 256 * 2 * ((BFGS_MAX_PAIRS + 15) / 16 + 1) * 16 * 2;
constexpr size_t kPartBytes = (size_t)80 << 20;                                          // 80 MiB
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kScratchBytes = align_up(kZBytes) + align_up(kPTBytes) + align_up(kSmall16Bytes) + kPartBytes;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on first use on that device).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BFGS_ERR_HIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return BFGS_ERR_HIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return BFGS_OK;
}

}  // namespace

extern "C" {

int bfgs_apply_Hinv_noalloc(bfgs_t h, const void* V, int32_t ncols, void* out) {
    if (!h || !V || !out || ncols < 1 || ncols > BFGS_MAX_COLS) return BFGS_ERR_ARG;
    if (V == out) return BFGS_ERR_ARG;
    if (h->gamma_mode && !h->gamma_known) return BFGS_ERR_STATE;
    // fixed parts sized for the largest handle; the partials' share bounds the split-K depth
    if ((size_t)2 * h->kmax * BFGS_MAX_COLS * sizeof(double) > kZBytes || apply_small16_bytes(h->kmax) > kSmall16Bytes)
        return BFGS_ERR_ARG;
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc != BFGS_OK) return rc;
    unsigned char* p = (unsigned char*)base;
    ApplyWs ws;
    ws.Z = (double*)p;
    p += align_up(kZBytes);
    ws.PT = (double*)p;
    p += align_up(kPTBytes);
    ws.small16 = (uint16_t*)p;
    p += align_up(kSmall16Bytes);
    ws.part = p;
    ws.part_bytes = kPartBytes;
    // no event pool may grow either: the call is not profiled
    const bool prof = h->prof.on;
    h->prof.on = false;
    rc = apply_block(h, V, ncols, out, false, false, &ws);
    h->prof.on = prof;
    return rc;
}

}  // extern "C"
