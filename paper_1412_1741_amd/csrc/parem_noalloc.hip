// parem_match_async_noalloc: parem_match_async with its workspace in a
// file-scope device array instead of a caller buffer, for callers that cannot
// allocate device memory. The array's device address is looked up once per
// device (hipGetSymbolAddress with that device current) and kept; host code
// uses only that address, never the array's name.
#include "parem_internal.h"

#include <mutex>

namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on first use)
parem_status scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return PAREM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PAREM_EDEVICE;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return PAREM_OK;
}

}  // namespace

extern "C" {

uint64_t parem_noalloc_scratch_bytes(void) { return kScratchBytes; }

parem_status parem_match_async_noalloc(parem_handle h, const uint8_t *d_text, uint64_t len, void *stream,
                                       parem_result *d_out) {
    if (!h || !d_out || (len && !d_text)) return PAREM_EINVAL;
    parem::PlainPlan p;
    parem_status st = parem::plan_plain(h->dev, len, &p);
    if (st != PAREM_OK) return st;
    if (p.bytes > kScratchBytes) return PAREM_EUNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PAREM_EDEVICE;
    if (dev != h->dev.device) return PAREM_EINVAL;  // the handle's tables live on its device
    void *ws = nullptr;
    st = scratch_ptr(dev, &ws);
    if (st != PAREM_OK) return st;
    return parem::launch_plain(h->dev, p, d_text, ws, reinterpret_cast<hipStream_t>(stream), d_out);
}

}  // extern "C"
