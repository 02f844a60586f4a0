// Internal definitions shared by the builder, the kernels and the C ABI.
#pragma once

#include <stdint.h>

#include <vector>

#include "lj.h"
#include "rmi_eval.h"

namespace lj {

// Slot of the gapped arrays of a gapped RMI (Section III-A, "GRMI
// Structure"): the key and its payload (the key's position in R) side by
// side, the gap bitmap folded into the payload, so that one 16-byte load
// reads all three.  A gap holds the next key of R (UINT64_MAX after the
// last one), which keeps the key array non-decreasing for the search.
struct alignas(16) GSlot {
    uint64_t key;
    uint32_t ridx;  // position in R, or kGap
    uint32_t pad;
};
constexpr uint32_t kGap = 0xFFFFFFFFu;

// Bucket of the learned hash index (Section III-C, "Learned-based Hash
// INLJ"): up to four keys of R with their positions, the number of keys
// held and the next bucket of the chain (kNoBucket at the end); one 64-byte
// line, read with four 16-byte loads.
struct alignas(64) HBucket {
    uint64_t key[4];
    uint32_t ridx[4];
    uint32_t next;
    uint32_t nkeys;
    uint32_t pad[2];
};
constexpr uint32_t kBucketSlots = 4;
constexpr uint32_t kNoBucket = 0xFFFFFFFFu;

}  // namespace lj

struct lj_index {
    uint64_t n = 0;
    uint32_t leaves = 0;
    uint32_t flags = 0;
    bool host_only = false;
    int device = -1;

    lj::RootModel root{};
    std::vector<uint32_t> root_tab;      // radix root: host copy (root.tab_host)
    uint32_t* root_tab_dev = nullptr;    // radix root: device copy (root.tab_dev)
    std::vector<lj::LeafF32> leaf32;  // host copy (LJ_LEAF_FP32)
    std::vector<lj::LeafF64> leaf64;  // host copy (LJ_LEAF_FP64)

    // statistics
    uint64_t max_mult = 0;
    uint32_t nonempty_leaves = 0;
    uint32_t max_leaf_keys = 0;
    double mean_window = 0.0;
    uint64_t max_window = 0;

    // LJ_PROBE_BINNED: kBins - 1 fences, fences[i] = R[(i + 1) * n / kBins]
    // (the bin of key x is the number of fences <= x), and per key bucket
    // the number of fences in lower buckets (kBuckets + 1 entries)
    std::vector<uint64_t> fences;
    std::vector<uint16_t> bucket_lo;

    // Gapped RMI: gap factor G (slots per key of R; 0 for a plain RMI), the
    // number of slots and the slot array (host copy kept for host-only
    // indexes).  A leaf's lo/hi then bound the slot of every key routed to it
    // relative to its predicted slot: 0 <= slot - predicted <= hi.
    uint32_t gap = 0;
    uint64_t nslots = 0;
    std::vector<lj::GSlot> slots;
    lj::GSlot* slots_dev = nullptr;

    // Learned hash index: slots per key of R (0 for none; buckets of four
    // slots), primary buckets (one per bucket value of the hash), all
    // buckets (primary, then overflow), the bucket array (host copy kept
    // for host-only indexes).
    uint32_t hash_spk = 0;
    uint64_t nprimary = 0;
    uint64_t nbuckets = 0;
    std::vector<lj::HBucket> buckets;
    lj::HBucket* buckets_dev = nullptr;

    // device copies
    uint64_t* r_dev = nullptr;
    // Line samples of R: rs[i] = R[kLineKeys * i], one key per 128-byte line
    // (the first stage of the binary search reads these, the second the one
    // line of R that holds the lower bound).
    uint64_t* rs_dev = nullptr;
    void* leaf_dev = nullptr;
    uint64_t* fences_dev = nullptr;
    uint16_t* bucket_lo_dev = nullptr;
    uint64_t device_bytes = 0;
};

namespace lj {

inline bool leaf_fp32(uint32_t flags) { return (flags & 3u) == LJ_LEAF_FP32; }

// Fit the root and leaf models and their error bounds on the host (no HIP
// calls).  Returns an LJ_* status.
int fit_rmi(const uint64_t* r, uint64_t n, uint32_t leaves, uint32_t flags,
            lj_index* idx);

// Turn a fitted RMI into a gapped RMI with G slots per key of R: model-based
// insertion of R into the slot array and per-leaf slot bounds (host only).
int fit_gapped(const uint64_t* r, uint32_t G, lj_index* idx);

// Build the learned hash index over a fitted RMI: every key of R, in order,
// appended to the chain of its bucket (host only).
int fit_hash(const uint64_t* r, uint32_t slots_per_key, lj_index* idx);

// Bucket of key x in a learned hash index: the leaf's predicted position,
// clamped into the leaf's run, times slots_per_key / kBucketSlots (the
// model's CDF estimate scaled to the primary buckets).  The leaf must not
// be empty.
template <class Leaf>
__host__ __device__ inline uint64_t hash_bucket(const Leaf& lf, uint64_t x, uint32_t spk) {
    int64_t rel = predict_rel(lf, x);
    if (rel < 0) rel = 0;
    if (rel > (int64_t)lf.cnt - 1) rel = (int64_t)lf.cnt - 1;
    return (((uint64_t)lf.pos0 + (uint64_t)rel) * spk) / kBucketSlots;
}

// Predicted slot of key x in a gapped index: the leaf's predicted position,
// clamped into the leaf's run, times G.  The leaf must not be empty.
template <class Leaf>
__host__ __device__ inline uint64_t gapped_pred(const Leaf& lf, uint64_t x, uint32_t G) {
    int64_t rel = predict_rel(lf, x);
    if (rel < 0) rel = 0;
    if (rel > (int64_t)lf.cnt - 1) rel = (int64_t)lf.cnt - 1;
    return ((uint64_t)lf.pos0 + (uint64_t)rel) * G;
}

// Tile geometry of the fused probe kernel: kBlock threads, each holding
// kItems outer keys.  Defaults: kItemsUnique when R has no duplicate keys,
// kItemsDup otherwise (at most kItemsDupMax: the LDS offsets per key),
// kItemsGapped on a gapped index, kItemsHash on a learned hash index; the
// shallowest depths that still keep enough loads in flight measured
// fastest.
constexpr int kBlock = 256;
constexpr uint32_t kLineKeys = 16;  // keys of R per 128-byte cache line (line samples)
// The direct probe searches in two stages when the index's mean window is at
// least this long (the binned probe always does).
constexpr double kTwoStageMinWindow = 64.0;
constexpr int kItemsUnique = 8;
constexpr int kItemsDup = 4;      // default with duplicates
constexpr int kItemsDupMax = 16;  // largest with duplicates (LDS offsets per key)
constexpr int kItemsGapped = 8;
constexpr int kItemsHash = 8;  // learned hash index: a 64-byte bucket in flight per key
constexpr int kItemsBinned = 16;  // search kernel of the binned probe (measured best)
constexpr int kItemsFused = 8;    // largest keys per lane of a fused launch
constexpr int kSetupChunk = 4;
constexpr int kMinTile = kBlock * 4;  // smallest tile any launch uses

// Workspace of a single probe: a 256-byte header followed by one status
// word per tile.
// The two counters every tile updates sit on separate cache lines: the
// device serialises updates of one line.
struct WsHeader {
    uint32_t tile_counter;  // dynamic tile ids
    uint32_t err;           // non-zero: a wait bound was hit
    uint32_t queue_count;   // binned probe of a gapped index: keys queued for the second pass
    uint32_t pad0;
    uint64_t count;         // total pairs (internal count slot)
    uint8_t pad1[128 - 24];
    uint32_t done_counter;  // tiles finished
};
static_assert(sizeof(WsHeader) <= 256, "header fits its 256 bytes");
constexpr uint64_t kWsHeaderBytes = 256;

inline uint64_t num_tiles(uint64_t m, uint64_t tile) { return (m + tile - 1) / tile; }
inline uint64_t align_up256(uint64_t v) { return (v + 255) & ~255ull; }
// Sized for the smallest tile, so one workspace fits every launch shape.
inline uint64_t ws_bytes_direct(uint64_t m) {
    return kWsHeaderBytes + num_tiles(m, kMinTile) * 8;
}

// Binned probe (LJ_PROBE_BINNED): S is put in key order of kBins equi-depth
// ranges of R by two stable partition passes over the two kDigitBits-bit
// digits of the bin number, probed in that order, and the results are put
// back in S order before emission.
constexpr uint32_t kBinBits = 12;
constexpr uint32_t kBins = 1u << kBinBits;  // kBins - 1 fences
constexpr uint32_t kDigitBits = 6;
constexpr uint32_t kDigits = 1u << kDigitBits;
static_assert(2 * kDigitBits == kBinBits, "two partition passes cover the bin number");
constexpr uint32_t kPartItems = 16;
constexpr uint32_t kPartChunk = kBlock * kPartItems;  // keys per partition chunk
constexpr uint32_t kScanTile = kBlock * 16;           // counts per scan tile
constexpr uint32_t kXcds = 8;  // workgroups are dealt to the XCDs round-robin

// Bucket of a key on a float-like scale (exponent and the next kBucketBits
// bits), monotone in the key.  The index keeps, per bucket, the number of
// fences in lower buckets, so a key's bin is found by searching only the
// few fences of its own bucket.
constexpr uint32_t kBucketBits = 8;
constexpr uint32_t kBuckets = (64 - kBucketBits + 1) << kBucketBits;  // 14592
__host__ __device__ inline uint32_t key_bucket(uint64_t x) {
    const int e = 63 - clz64(x | 1);  // floor(log2 x); 0 for x <= 1
    const uint32_t hi = ((uint32_t)(e - (int)kBucketBits + 1) << kBucketBits) |
                        (uint32_t)((x >> (e >= (int)kBucketBits ? e - (int)kBucketBits : 0)) &
                                   ((1u << kBucketBits) - 1));
    return x < (1ull << kBucketBits) ? (uint32_t)x : hi;
}

// Byte offsets inside the workspace of a binned probe.  [0, ctrl_bytes) is
// zeroed before every probe: the header (error flag), the counter block
// (scan tile counters in words 0-1, the emission's tile counter in word 2
// and its done counter in word 32, a cache line further), the scans'
// status words and one word per chunk of S (the emission's look-back
// words; the sort join keeps per-chunk pair counts there).  res2/res1 (per-key results
// in bin and pass-1 order) reuse p1 and p2 once those are dead.
struct BinnedWs {
    uint64_t scan_ctr, scan_st1, scan_st2, scan_st3, counts, ctrl_bytes;
    uint64_t hist1, hist2, bins_s, bins_1, p1, p2, dest1, dest2, total;
};
inline BinnedWs binned_ws(uint64_t m) {
    BinnedWs L{};
    const uint64_t nchunks = num_tiles(m, kPartChunk);
    const uint64_t nh = (uint64_t)kDigits * nchunks;
    const uint64_t nscan = num_tiles(nh, kScanTile);
    uint64_t a = kWsHeaderBytes;
    L.scan_ctr = a;
    a += 256;
    L.scan_st1 = a;
    a = align_up256(a + nscan * 8);
    L.scan_st2 = a;
    a = align_up256(a + nscan * 8);
    L.scan_st3 = a;
    a = align_up256(a + num_tiles(nchunks + 1, kScanTile) * 8);
    L.counts = a;  // pairs per chunk of S, then their exclusive prefix (+ total)
    a = align_up256(a + (nchunks + 1) * 8);
    L.ctrl_bytes = a;
    L.hist1 = a;
    a = align_up256(a + nh * 4);
    L.hist2 = a;
    a = align_up256(a + nh * 4);
    L.bins_s = a;
    a = align_up256(a + m * 2);
    L.bins_1 = a;
    a = align_up256(a + m * 2);
    L.p1 = a;
    a = align_up256(a + m * 8);
    L.p2 = a;
    a = align_up256(a + m * 8);
    L.dest1 = a;
    a = align_up256(a + m * 4);
    L.dest2 = a;
    a = align_up256(a + m * 4);
    L.total = a;
    return L;
}
// Probe form: mode < 0 follows the index's LJ_PROBE_BINNED flag, 0 is the
// direct probe, > 0 the binned probe (when R is not empty).
inline bool uses_binned(const lj_index* idx, uint64_t m, int mode = -1) {
    const bool want = mode < 0 ? (idx->flags & LJ_PROBE_BINNED) != 0 : mode > 0;
    return want && idx->n > 0 && m > 0 && !idx->fences.empty();
}
// Workspace of one probe of m keys against idx.
inline uint64_t ws_bytes(const lj_index* idx, uint64_t m, int mode = -1) {
    return uses_binned(idx, m, mode) ? binned_ws(m).total : ws_bytes_direct(m);
}

// Everything the device needs to probe the tiles of one batch of outer keys
// against one index.
struct TileJob {
    const uint64_t* r;
    const uint64_t* rs;    // line samples of R
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
    uint32_t kind;         // kJobFp64 | kJobDup | kJobExp | kJobGapped | kJobHash
    uint32_t kpl;          // keys per lane in this batch's tiles
    const GSlot* slots;    // gapped index: slot array, its size and gap factor
    uint32_t nslots;
    uint32_t gap;
    const HBucket* buckets;  // learned hash index: buckets, slots per key
    uint32_t hash_spk;
};
constexpr uint32_t kJobFp64 = 1u;
constexpr uint32_t kJobDup = 2u;
constexpr uint32_t kJobExp = 4u;
constexpr uint32_t kJobGapped = 8u;
constexpr uint32_t kJobHash = 16u;

inline uint32_t job_kind(const lj_index* idx) {
    return ((idx->flags & LJ_LEAF_FP64) ? kJobFp64 : 0u) | (idx->max_mult > 1 ? kJobDup : 0u) |
           ((idx->flags & LJ_SEARCH_EXPONENTIAL) ? kJobExp : 0u) |
           (idx->gap ? kJobGapped : 0u) | (idx->hash_spk ? kJobHash : 0u);
}

// One batch of a fused launch (many batches, one kernel): the
// batch's job, the id of its first tile in the launch's shared tile-id
// space, and whether its search takes the line-sample stage.  Each batch
// has a workspace of fused_job_ws_bytes(m, kpl): a done counter, then one
// look-back status word per tile; the launch shares a kFusedHeader-byte
// header (tile counter, error flag), which err points into.
struct FusedJob {
    TileJob j;
    uint32_t tile0;
    uint32_t two_stage;
    uint64_t pad;
};
constexpr uint64_t kFusedJobHeader = 256;
constexpr uint64_t kFusedHeader = 256;  // word 0: tile counter, word 1: error flag
inline uint64_t fused_job_ws_bytes(uint64_t m, uint32_t kpl) {
    return kFusedJobHeader + num_tiles(m, (uint64_t)kBlock * kpl) * 8;
}

// Kernel launchers (lj_kernels.hip).  Return hipSuccess or the launch error.
// kpl: keys per lane of the launch (4, 8, 16 or, without duplicates, 24;
// 0 = the default for the index).
bool probe_kpl_supported(uint32_t kpl, bool dup);
// Fused launches: the kernel group of an index (0..kFusedGroups-1: leaf
// arithmetic, duplicates, plain or gapped RMI; -1 for index kinds a fused
// launch does not take: learned hash, exponential search), the keys per
// lane a batch gets in it, one batch's entry, and the launch itself (clears
// the header and every batch's workspace first; jobs_dev in device memory,
// sorted by tile0, all of group `group`).
constexpr int kFusedGroupGapped = 4;  // + (kJobFp64 | kJobDup) bits
constexpr int kFusedGroups = 8;
int fused_group(const lj_index* idx);
uint32_t fused_kpl(const lj_index* idx, uint32_t kpl);
FusedJob make_fused_job(const lj_index* idx, const uint64_t* s, uint64_t m, lj_pair* out,
                        uint64_t cap, uint64_t* count_out, void* job_ws, uint32_t kpl,
                        uint32_t* err, uint32_t tile0);
hipError_t launch_probe_fused(const FusedJob* jobs_dev, uint32_t njobs, uint32_t total_tiles,
                              int group, uint32_t* hdr, hipStream_t stream);
hipError_t launch_probe(const lj_index* idx, const uint64_t* s, uint64_t m,
                        lj_pair* out, uint64_t cap, uint64_t* count_dev,
                        void* ws, hipStream_t stream, hipEvent_t ev0,
                        hipEvent_t ev1, uint32_t kpl = 0,  // kpl: direct probe only
                        int mode = -1);                    // see uses_binned
// Binned probe pieces (lj_partition.hip): the two partition passes of S
// into the workspace laid out by binned_ws(m); out[p] = in[dest[p]] over m
// elements of 4 bytes (8 with `wide`); the same with the number of pairs of
// each chunk of kPartChunk outputs added to counts[chunk] (4-byte elements:
// 1 unless ~0u; 8-byte: the high word), followed by the exclusive prefix of
// counts[0 .. nchunks] in place, so counts[nchunks] = total.
hipError_t launch_partition(const lj_index* idx, const uint64_t* s, uint64_t m, void* ws,
                            const BinnedWs& layout, hipStream_t stream);
hipError_t launch_unpermute(const uint32_t* dest, const void* in, void* out, uint64_t m,
                            bool wide, hipStream_t stream);
hipError_t launch_unpermute_count(const uint32_t* dest, const void* in, void* out, uint64_t m,
                                  bool wide, void* ws, const BinnedWs& layout,
                                  hipStream_t stream);
hipError_t launch_set_u64(uint64_t* p, uint64_t v, hipStream_t stream);
// In-place exclusive prefix sum of n uint32 counts (total < 2^32); status:
// num_tiles(n, kScanTile) zeroed words, ctr: a zeroed counter.
hipError_t launch_scan_u32(uint32_t* d, uint64_t n, uint64_t* status, uint32_t* ctr,
                           uint32_t* err, hipStream_t stream);

// rs[i] = r[kLineKeys * i] for i < ceil(n / kLineKeys).
hipError_t launch_line_samples(const uint64_t* r, uint64_t n, uint64_t* rs, hipStream_t stream);
hipError_t launch_zero_words(uint64_t* p, uint64_t nwords, hipStream_t stream);
// violations_dev: two words (the count, then scratch for a gapped index).
hipError_t launch_self_check(const lj_index* idx, uint64_t* violations_dev,
                             hipStream_t stream);
hipError_t launch_predict_windows(const lj_index* idx, const uint64_t* keys,
                                  uint64_t m, uint32_t* leaf, int64_t* pred,
                                  int64_t* wlo, int64_t* whi, hipStream_t stream);
hipError_t launch_random_gather(const void* buf, uint64_t bytes, uint32_t granule,
                                uint64_t reads, uint64_t seed, uint64_t* sink,
                                hipStream_t stream);

}  // namespace lj
