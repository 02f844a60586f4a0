// Internal definitions shared by the builder, the kernels and the C ABI.
#pragma once

#include <stdint.h>

#include <vector>

#include "lj.h"
#include "rmi_eval.h"

struct lj_index {
    uint64_t n = 0;
    uint32_t leaves = 0;
    uint32_t flags = 0;
    bool host_only = false;
    int device = -1;

    lj::RootModel root{};
    std::vector<lj::LeafF32> leaf32;  // host copy (LJ_LEAF_FP32)
    std::vector<lj::LeafF64> leaf64;  // host copy (LJ_LEAF_FP64)

    // statistics
    uint64_t max_mult = 0;
    uint32_t nonempty_leaves = 0;
    uint32_t max_leaf_keys = 0;
    double mean_window = 0.0;
    uint64_t max_window = 0;

    // device copies
    uint64_t* r_dev = nullptr;
    void* leaf_dev = nullptr;
    uint64_t device_bytes = 0;
};

namespace lj {

inline bool leaf_fp32(uint32_t flags) { return (flags & 3u) == LJ_LEAF_FP32; }

// Fit the root and leaf models and their error bounds on the host (no HIP
// calls).  Returns an LJ_* status.
int fit_rmi(const uint64_t* r, uint64_t n, uint32_t leaves, uint32_t flags,
            lj_index* idx);

// Tile geometry of the fused probe kernel: kBlock threads, each holding
// kItems outer keys (kItemsUnique when R has no duplicate keys, kItemsDup
// otherwise, where the run scan and the LDS offsets need more room).
constexpr int kBlock = 256;
constexpr int kItemsUnique = 24;
constexpr int kItemsDup = 16;
constexpr int kSetupChunk = 4;
constexpr int kMinTile = kBlock * 4;  // smallest tile any launch uses

// Workspace of a single probe: a 256-byte header followed by one status
// word per tile.
struct WsHeader {
    uint32_t tile_counter;  // dynamic tile ids
    uint32_t done_counter;  // tiles finished
    uint32_t err;           // non-zero: a wait bound was hit
    uint32_t pad0;
    uint64_t count;         // total pairs (internal count slot)
};
constexpr uint64_t kWsHeaderBytes = 256;

inline uint64_t num_tiles(uint64_t m, uint64_t tile) { return (m + tile - 1) / tile; }
// Sized for the smallest tile, so one workspace fits every launch shape.
inline uint64_t ws_bytes(uint64_t m) { return kWsHeaderBytes + num_tiles(m, kMinTile) * 8; }

// Everything the device needs to probe the tiles of one batch of outer keys
// against one index.
struct TileJob {
    const uint64_t* r;
    const void* leaves;
    RootModel root;
    const uint64_t* s;
    uint64_t m;
    lj_pair* out;
    uint64_t cap;          // 0 when out is null
    uint64_t* count_out;   // receives the batch's total (UINT64_MAX on error)
    uint64_t* status;      // ntiles look-back words
    uint32_t* done;        // tiles of this batch finished
    uint32_t* err;         // error flag shared by the launch
    uint32_t ntiles;
    uint32_t kind;         // kJobFp64 | kJobDup
    uint32_t kpl;          // keys per lane in this batch's tiles
};
constexpr uint32_t kJobFp64 = 1u;
constexpr uint32_t kJobDup = 2u;
constexpr uint32_t kJobExp = 4u;

inline uint32_t job_kind(const lj_index* idx) {
    return ((idx->flags & LJ_LEAF_FP64) ? kJobFp64 : 0u) | (idx->max_mult > 1 ? kJobDup : 0u) |
           ((idx->flags & LJ_SEARCH_EXPONENTIAL) ? kJobExp : 0u);
}

// Kernel launchers (lj_kernels.hip).  Return hipSuccess or the launch error.
// kpl: keys per lane of the launch (4, 8, 16 or, without duplicates, 24;
// 0 = the default for the index).
bool probe_kpl_supported(uint32_t kpl, bool dup);
hipError_t launch_probe(const lj_index* idx, const uint64_t* s, uint64_t m,
                        lj_pair* out, uint64_t cap, uint64_t* count_dev,
                        void* ws, hipStream_t stream, hipEvent_t ev0,
                        hipEvent_t ev1, uint32_t kpl = 0);
hipError_t launch_set_u64(uint64_t* p, uint64_t v, hipStream_t stream);
hipError_t launch_zero_words(uint64_t* p, uint64_t nwords, hipStream_t stream);
hipError_t launch_self_check(const lj_index* idx, uint64_t* violations_dev,
                             hipStream_t stream);
hipError_t launch_predict_windows(const lj_index* idx, const uint64_t* keys,
                                  uint64_t m, uint32_t* leaf, int64_t* pred,
                                  int64_t* wlo, int64_t* whi, hipStream_t stream);
hipError_t launch_random_gather(const void* buf, uint64_t bytes, uint32_t granule,
                                uint64_t reads, uint64_t seed, uint64_t* sink,
                                hipStream_t stream);

}  // namespace lj
