// Learned sort join (Section IV): workspace layout and launchers.
#pragma once

#include "lj_internal.h"

namespace lj {

// Learned sort join (Section IV).  The CDF model of R is a linear spline
// over equi-depth knots of a sorted sample of R (kSjSamples keys sorted in
// one block's LDS, one knot per kSjSamplesPerKnot samples), located through
// the key bucket table.  Scaled by `fan` sub-partitions per segment it
// gives every key a partition number (pid), monotone in the key, over
// (nk + 2) * fan partitions: fan over [0, first knot), fan per knot
// segment, fan from the last knot k on (over [k, 2k), keys beyond in the
// last).  R is put in pid order by stable partition passes (kDigitBits bits
// each, payload: the input position), then every partition is sorted by
// (key, position): by one wave in registers up to 2048 keys, by a block in
// LDS up to kSjSortCap, beyond that by a larger block (in LDS, or in
// global memory).  S is put in coarse pid order by two passes and each key
// is found in its own partition of the sorted R.
constexpr uint32_t kSjSamples = 16384;
constexpr uint32_t kSjSamplesPerKnot = 16;
constexpr uint32_t kSjMaxSegments = kSjSamples / kSjSamplesPerKnot - 2;
constexpr uint32_t kSjTargetPart = 1024;  // mean keys per partition of R at most this
constexpr uint32_t kSjMaxFan = 256;
constexpr uint32_t kSjSortCap = 4096;
constexpr uint32_t kSjMaxPasses = 4;
struct SortJoinWs {
    uint32_t ns, nk, fan, parts, nbits, rpasses, spasses, s_shift;
    uint64_t scan_ctr, scan_st[kSjMaxPasses + 3], counts, big_queue, ctrl_bytes;
    uint64_t knots, kb_lo, r_hist, r_bins[2], r_keys[2], r_pos[2], r_start, r_rs;
    uint64_t s_hist, s_bins[2], s_keys[2], s_dest[2], total;
};
inline SortJoinWs sort_join_ws(uint64_t n, uint64_t m) {
    SortJoinWs L{};
    L.ns = n < kSjSamples ? (uint32_t)n : kSjSamples;
    L.nk = L.ns / kSjSamplesPerKnot > 2 ? L.ns / kSjSamplesPerKnot - 2 : 1;
    const uint64_t want = num_tiles(n, (uint64_t)(L.nk + 2) * kSjTargetPart);
    L.fan = 1;
    while (L.fan < want && L.fan < kSjMaxFan) L.fan <<= 1;
    L.parts = (L.nk + 2) * L.fan;
    while ((1ull << L.nbits) < L.parts) ++L.nbits;
    L.rpasses = L.nbits ? (L.nbits + kDigitBits - 1) / kDigitBits : 1;
    L.spasses = 2;
    L.s_shift = L.nbits > 2 * kDigitBits ? L.nbits - 2 * kDigitBits : 0;
    const uint64_t nchr = num_tiles(n, kPartChunk), nchs = num_tiles(m, kPartChunk);
    const uint64_t nhr = (uint64_t)kDigits * nchr, nhs = (uint64_t)kDigits * nchs;
    uint64_t a = kWsHeaderBytes;
    L.scan_ctr = a;  // 64 tile counters
    a += 256;
    for (uint32_t k = 0; k < kSjMaxPasses + 3; ++k) {
        const uint64_t tiles = k < kSjMaxPasses       ? num_tiles(nhr, kScanTile)
                               : k < kSjMaxPasses + 2 ? num_tiles(nhs, kScanTile)
                                                      : num_tiles(nchs + 1, kScanTile);
        L.scan_st[k] = a;
        a = align_up256(a + tiles * 8);
    }
    L.counts = a;  // pairs per chunk of S, then their exclusive prefix (+ total)
    a = align_up256(a + (nchs + 1) * 8);
    L.big_queue = a;  // count, the partitions too large for LDS, the join's run flag
    a = align_up256(a + 8 + (uint64_t)L.parts * 4);
    L.ctrl_bytes = a;
    L.knots = a;
    a = align_up256(a + (uint64_t)(L.nk + 1) * 8);
    L.kb_lo = a;
    a = align_up256(a + (uint64_t)(kBuckets + 1) * 2);
    L.r_hist = a;
    a = align_up256(a + nhr * 4);
    for (int k = 0; k < 2; ++k) {
        L.r_bins[k] = a;
        a = align_up256(a + n * 4);
        L.r_keys[k] = a;
        a = align_up256(a + n * 8);
        L.r_pos[k] = a;
        a = align_up256(a + n * 4);
    }
    L.r_start = a;
    a = align_up256(a + ((uint64_t)L.parts + 1) * 4);
    L.r_rs = a;  // line samples of the sorted R
    a = align_up256(a + num_tiles(n, kLineKeys) * 8);
    L.s_hist = a;
    a = align_up256(a + nhs * 4);
    for (int k = 0; k < 2; ++k) {
        L.s_bins[k] = a;
        a = align_up256(a + m * 4);
        L.s_keys[k] = a;
        a = align_up256(a + m * 8);
        L.s_dest[k] = a;
        a = align_up256(a + m * 4);
    }
    L.total = a;
    return L;
}

// The learned sort of n keys into (key, position) order (keys_out/pos_out:
// caller buffers, or null for the workspace's own) and the whole join, in a
// workspace laid out by sort_join_ws(n, m) (lj_sortjoin.hip).
hipError_t launch_learned_sort(const uint64_t* keys, uint64_t n, uint64_t* keys_out,
                               uint32_t* pos_out, void* ws, const SortJoinWs& layout,
                               hipStream_t stream);
hipError_t launch_sort_join(const uint64_t* r, uint64_t n, const uint64_t* s, uint64_t m,
                            lj_pair* out, uint64_t cap, uint64_t* count_dev, void* ws,
                            hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);

}  // namespace lj
