// Probe entry point that allocates nothing: the direct probe with its
// workspace (tile counter, done counter, error flag and one look-back status
// word per tile) in a fixed device array owned by the library instead of a
// caller buffer or a hipMalloc.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lj_internal.h"

namespace {

// Room for the direct probe's workspace of up to kNoAllocMaxKeys outer keys
// (header + one 8-byte status word per 1024-key tile, the smallest tile).
constexpr uint64_t kNoAllocScratchBytes = 4ull << 20;
constexpr uint64_t kNoAllocMaxKeys =
    ((kNoAllocScratchBytes - lj::kWsHeaderBytes) / 8) * (uint64_t)lj::kMinTile;
static_assert(lj::kMinTile == 1024, "workspace sizing assumes 1024-key tiles");

// One copy per GPU, held until the process ends.  Host code never passes
// this name to a kernel: it is a host-side stand-in; the device address of
// each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return LJ_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return LJ_ERR_DEVICE;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return LJ_OK;
}

}  // namespace

extern "C" {

uint64_t lj_probe_join_noalloc_max_keys(void) { return kNoAllocMaxKeys; }

int lj_probe_join_noalloc(const lj_index* idx, const uint64_t* s, uint64_t m, lj_pair* out,
                          uint64_t cap, uint64_t* count_dev, hipStream_t stream) {
    if (!idx || idx->host_only || !count_dev) return LJ_ERR_ARG;
    if (m > 0 && !s) return LJ_ERR_ARG;
    if (cap > 0 && !out) return LJ_ERR_ARG;
    if (m > kNoAllocMaxKeys) return LJ_ERR_TOO_LARGE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LJ_ERR_DEVICE;
    if (dev != idx->device) return LJ_ERR_ARG;
    if (m == 0)
        return lj::launch_set_u64(count_dev, 0, stream) == hipSuccess ? LJ_OK : LJ_ERR_DEVICE;
    void* ws = nullptr;
    const int st = scratch_ptr(dev, &ws);
    if (st != LJ_OK) return st;
    // The direct probe (mode 0): its workspace does not grow with the keys'
    // results, so it fits the fixed array; launch_probe clears it with a
    // kernel before the probe.
    if (lj::ws_bytes_direct(m) > kNoAllocScratchBytes) return LJ_ERR_TOO_LARGE;
    const hipError_t e = lj::launch_probe(idx, s, m, out, cap, count_dev, ws, stream, nullptr,
                                          nullptr, 0, 0);
    return e == hipSuccess ? LJ_OK : LJ_ERR_DEVICE;
}

}  // extern "C"
