// The allocation-free variant of the Frank-Wolfe solve, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops
// that keep the allocator out of the steady state).
//
// Its per-call buffers live in one file-scope device array, `scratch`, of
// kScratchBytes. In host code the array's name is only a host-side handle:
// its device address, which differs on every device, comes from
// hipGetSymbolAddress, taken once per device (with that device current) at
// the entry point's first call on it and kept in g_scratch; kernels receive
// that address. Every call on one device shares the array, which keeps the
// last call's contents: the solve clears what must start at zero itself, and
// calls that overlap on one device (two streams, two threads) race.

#include <mutex>

#include "dcrf_internal.h"

namespace dcrf {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// the device address of `scratch` on `device` (the current device)
void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices)
        fail(DCRF_EUNSUPPORTED, "device index beyond the allocation-free scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        DCRF_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[device] = p;
    }
    return g_scratch[device];
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

void frank_wolfe_noalloc_entry(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                               void *y, int iters, dcrf_iter_trace *trace) {
    frank_wolfe_noalloc(ctx, unary, mu, L, y, iters, trace, scratch_address(ctx->device),
                        kScratchBytes);
}

}  // namespace dcrf
