// GPU kernels of the learned indexed nested loop join probe (gfx950).
//
// One fused kernel runs the whole probe for a tile of outer keys
// (Section II-A: scan S, use the index on R to fetch the tuples with the same
// key; Section II-D: root model -> leaf model -> bounded last-mile search;
// Section VI-B, "Duplicates": range scan of equal keys inside the bounds):
//
//   1. coalesced read of the tile's S keys (lane t of the block handles keys
//      t, t+256, t+512, t+768 of the tile);
//   2. root model (FP64 fma) -> leaf record (32 or 48 bytes, read through
//      L2/MALL) -> leaf model (FP32 fmaf or FP64 fma) -> window [lo, hi];
//   3. lower_bound in R over the window, the kItems keys of a lane advanced
//      in lockstep so that each lane keeps kItems independent loads in flight,
//      in two stages (the window's line samples, one key per 128-byte line
//      of R, then the candidate positions of one line); the element found is
//      the last one read with value >= x, so the equality test needs no
//      extra load.  On a gapped index the search gallops forward from the
//      predicted slot instead, and on a learned hash index it walks the
//      bucket chain;
//   4. length of the run of equal keys (only when R has duplicates);
//   5. tile-local exclusive offsets of the outputs: ballot/popcount per wave
//      when every count is 0 or 1, an LDS scan otherwise;
//   6. global offset of the tile by a single-pass decoupled look-back over the
//      tiles' status words (Merrill and Garland, "Single-pass parallel prefix
//      scan with decoupled look-back", NVIDIA TR 2016), tile ids handed out
//      by an atomic counter so that every predecessor of a waiting tile is
//      already running;
//   7. pair emission in (s_idx, r_idx) order: one store per match when every
//      count is 0 or 1, otherwise a load-balanced loop in which each output
//      slot finds its key by binary search over the LDS offsets, so stores
//      stay contiguous for any run length.
//
// No S key, count or offset makes a round trip through HBM between the
// steps: the only traffic is S, the R lines and leaf records the searches
// touch, the pairs, and 8 bytes of status per tile.
#include <hip/hip_runtime.h>

#include "lj_device.h"
#include "lj_internal.h"

namespace lj {
namespace {

// Leaf records are read as whole 16-byte vectors.
__device__ inline LeafF32 leaf_from(const uint4& a, const uint4& b) {
    LeafF32 l;
    l.base = (uint64_t)a.x | ((uint64_t)a.y << 32);
    l.slope = __uint_as_float(a.z);
    l.icpt = __uint_as_float(a.w);
    l.pos0 = b.x;
    l.cnt = b.y;
    l.lo = (int32_t)b.z;
    l.hi = (int32_t)b.w;
    return l;
}

__device__ inline LeafF32 load_leaf(const LeafF32* p) {
    const uint4* q = (const uint4*)p;
    return leaf_from(q[0], q[1]);
}

__device__ inline LeafF64 leaf_from(const uint4& a, const uint4& b, const uint4& c) {
    LeafF64 l;
    l.base = (uint64_t)a.x | ((uint64_t)a.y << 32);
    l.slope = __hiloint2double((int)a.w, (int)a.z);
    l.icpt = __hiloint2double((int)b.y, (int)b.x);
    l.pos0 = b.z;
    l.cnt = b.w;
    l.lo = (int32_t)c.x;
    l.hi = (int32_t)c.y;
    l.pad = 0;
    return l;
}

__device__ inline LeafF64 load_leaf(const LeafF64* p) {
    const uint4* q = (const uint4*)p;
    return leaf_from(q[0], q[1], q[2]);
}

// Radix root table in LDS: every thread block that routes keys copies the
// table (15 KB, kRootTabLen words, a multiple of 4) once, so the two table
// reads of each routing are LDS reads.  Linear roots need no table.
__device__ __forceinline__ void stage_root(const RootModel& rm, uint32_t* lds) {
    if (rm.kind != kRootRadix) return;
    const uint4* src = (const uint4*)rm.tab_dev;
    uint4* dst = (uint4*)lds;
    for (uint32_t i = threadIdx.x; i < kRootTabLen / 4; i += blockDim.x) dst[i] = src[i];
}

__device__ __forceinline__ uint32_t route_lds(const RootModel& rm, const uint32_t* lds,
                                              uint64_t x) {
    return rm.kind == kRootRadix ? route_radix(rm, lds, x) : route(rm, x);
}

// Shared memory of one tile; the duplicate path needs the per-key offsets
// and first positions, the unique path only the per-wave counts.
template <int kItems, bool kWithOffsets>
struct TileShared {
    uint64_t excl;
    uint64_t wsum[kItems * (kBlock / 64)];
    uint64_t off[kWithOffsets ? kBlock * kItems + 1 : 1];
    uint32_t j0[kWithOffsets ? kBlock * kItems : 1];
};

// Last tile of a batch to finish writes the batch's total (or UINT64_MAX
// after a wait error).  No fence orders a tile's status word before its
// count of finished tiles (an agent-scope fence writes back the whole L2
// and cost more than the rest of a short tile); instead the last tile to
// finish waits until the inclusive prefix of the batch's last tile is
// visible.  Every tile stored its inclusive prefix before counting itself
// as done, so the wait ends; a wait error was flagged with a sequentially
// consistent update before the flagging tile counted itself.
__device__ void finish_tile(const TileJob& j) {
    if (threadIdx.x == 0) {
        uint32_t done = atomicAdd(j.done, 1u);
        if (done == j.ntiles - 1) {
            const uint64_t* last = &j.status[j.ntiles - 1];
            uint64_t st = ld_status(last);
            for (uint32_t spins = 0; (st >> 62) != 2 && spins < kSpinLimit; ++spins) {
                __builtin_amdgcn_s_sleep(1);
                st = ld_status(last);
            }
            uint32_t e = __hip_atomic_load(j.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *j.count_out = e || (st >> 62) != 2 ? ~0ull : st & kValMask;
            // The count may live in pinned host memory (serving loop).
            __threadfence_system();
        }
    }
}

// Lockstep lower_bound over array A for the kItems keys of a lane: key k
// searches [first[k], first[k] + len[k]).  Finished keys re-read A[0] (a
// cached line) so that the loop body has no branches and the loads of all
// keys issue back to back.  On return first[k] is the range's end or the
// position of the last element read with A[mid] >= x[k], and bit k of
// eqmask tells whether that element equals x[k] (unchanged when no element
// >= x[k] was read).
template <int kItems>
__device__ __forceinline__ void bisect_lockstep(const uint64_t* __restrict__ A,
                                                const uint64_t (&x)[kItems],
                                                uint32_t (&first)[kItems],
                                                uint32_t (&len)[kItems], uint32_t& eqmask) {
    for (;;) {
        uint32_t anylen = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) anylen |= len[k];
        if (!anylen) break;
        uint64_t v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = A[len[k] ? first[k] + (len[k] >> 1) : 0];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t half = len[k] >> 1;
            const uint32_t act = len[k] != 0 ? 1u : 0u;
            const uint32_t lt = v[k] < x[k] ? act : 0u;   // act && lt
            const uint32_t ge = act ^ lt;                   // act && !lt
            const uint32_t eq = v[k] == x[k] ? 1u : 0u;
            first[k] += lt * (half + 1);
            eqmask = (eqmask & ~(ge << k)) | ((eq & ge) << k);
            len[k] = lt ? len[k] - half - 1 : half;
        }
    }
}

// Steps 1-4 for the keys of one tile: kBlock threads, the first `kpl`
// (<= kItems) keys of each lane are live; key k of thread t is
// s[tbase + k*kBlock + t].  On return first[k] is the lower bound of the key
// in R (inside its window) and c[k] the number of R keys equal to it (0 for
// a miss or a key past the end of s).
template <class Leaf, bool kUnique, int kItems, bool kExp, bool kTwoStage = true>
__device__ __forceinline__ void search_keys(const uint64_t* __restrict__ R,
                                            const uint64_t* __restrict__ RS, const Leaf* leaves,
                                            const RootModel& root, const uint32_t* rtab,
                                            const uint64_t* s,
                                            const uint64_t m, const uint64_t tbase,
                                            const uint32_t kpl, uint32_t (&first)[kItems],
                                            uint32_t (&c)[kItems],
                                            const bool two_stage = kTwoStage) {
    const int tid = threadIdx.x;
    uint64_t x[kItems];
    uint32_t len[kItems];  // binary search: window length
    int32_t lo[kExp ? kItems : 1], hi[kExp ? kItems : 1];  // exponential search:
    uint32_t pos[kExp ? kItems : 1], stp[kExp ? kItems : 1];  // bracket, probe, step|phase
    uint32_t end[kUnique ? 1 : kItems];
    uint32_t eqmask = 0;  // bit k: the last R[mid] >= x[k] read equals x[k]
    static_assert(kItems <= 32, "eqmask holds one bit per key");

    // 1: keys.  Loads are unconditional (clamped index) so that all the
    // loads of a lane are in flight together.
    uint32_t validmask = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = tbase + (uint64_t)k * kBlock + tid;
        const bool ok = (uint32_t)k < kpl && q < m;
        validmask |= (ok ? 1u : 0u) << k;
        x[k] = s[ok ? q : m - 1];
    }
    // 2: root model, leaf record, leaf model, window; kSetupChunk records
    // in flight at a time to bound register use.
#pragma unroll
    for (int k0 = 0; k0 < kItems; k0 += kSetupChunk) {
        Leaf lf[kSetupChunk];
#pragma unroll
        for (int u = 0; u < kSetupChunk; ++u)
            lf[u] = load_leaf(leaves + route_lds(root, rtab, x[k0 + u]));
#pragma unroll
        for (int u = 0; u < kSetupChunk; ++u) {
            const int k = k0 + u;
            int64_t rel = predict_rel(lf[u], x[k]);
            int64_t wlo = rel + lf[u].lo, whi = rel + lf[u].hi;
            if (wlo < 0) wlo = 0;
            if (whi > (int64_t)lf[u].cnt - 1) whi = (int64_t)lf[u].cnt - 1;
            const bool live = ((validmask >> k) & 1u) && lf[u].cnt != 0 && wlo <= whi;
            if constexpr (kExp) {
                // Open bracket (lo, hi) around the window; the first probe is
                // the prediction itself, clamped into the window.
                const int32_t a = (int32_t)lf[u].pos0 + (int32_t)wlo;
                const int32_t b = (int32_t)lf[u].pos0 + (int32_t)whi;
                int32_t pr = (int32_t)lf[u].pos0 + (int32_t)rel;
                pr = pr < a ? a : (pr > b ? b : pr);
                lo[k] = live ? a - 1 : 0;
                hi[k] = live ? b + 1 : 0;
                pos[k] = live ? (uint32_t)pr : 0;
                stp[k] = 0;  // phase 0: probe the prediction
            } else {
                first[k] = live ? lf[u].pos0 + (uint32_t)wlo : 0;
                len[k] = live ? (uint32_t)(whi - wlo + 1) : 0;
            }
            if constexpr (!kUnique) end[k] = live ? lf[u].pos0 + (uint32_t)whi + 1 : 0;
        }
    }

    if constexpr (kExp) {
        // 3': lockstep exponential search from the prediction, bounded by the
        // window.  The bracket (lo, hi) always satisfies R[lo] < x <= R[hi]
        // (positions a-1 and b+1 standing for the window's edges).  Phase 0
        // reads the prediction; phase 1 (2) gallops right (left) with steps
        // 8, 16, 32, ...; phase 3 bisects the bracket.  A key is done when
        // hi - lo <= 1; hi is then the lower bound and the last probe that
        // set hi tells whether x was found.
        for (;;) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < kItems; ++k) any |= hi[k] - lo[k] > 1;
            if (!any) break;
            uint64_t v[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k) v[k] = R[hi[k] - lo[k] > 1 ? pos[k] : 0];
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                if (hi[k] - lo[k] <= 1) continue;
                const uint32_t phase = stp[k] & 7u;
                uint32_t lg = stp[k] >> 3;  // step = 2^lg
                const bool lt = v[k] < x[k];
                if (lt) lo[k] = (int32_t)pos[k];
                else {
                    hi[k] = (int32_t)pos[k];
                    eqmask = (eqmask & ~(1u << k)) | ((v[k] == x[k] ? 1u : 0u) << k);
                }
                uint32_t nphase = phase;
                if (phase == 0) {
                    nphase = lt ? 1u : 2u;
                    lg = 3;
                } else if (phase == 1) {
                    if (lt) lg = lg < 30 ? lg + 1 : 30;
                    else nphase = 3;
                } else if (phase == 2) {
                    if (!lt) lg = lg < 30 ? lg + 1 : 30;
                    else nphase = 3;
                }
                stp[k] = (lg << 3) | nphase;
                const uint32_t step = 1u << lg;
                const int32_t l = lo[k], h = hi[k];
                int32_t np;
                if (nphase == 1) np = (int64_t)l + step < h - 1 ? l + (int32_t)step : h - 1;
                else if (nphase == 2) np = (int64_t)h - step > l + 1 ? h - (int32_t)step : l + 1;
                else np = l + ((h - l) >> 1);
                pos[k] = (uint32_t)np;
            }
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) first[k] = (uint32_t)hi[k];
    } else {
        // 3: lockstep lower_bound over the windows (bisect_lockstep), in two
        // stages (below).
        // Two stages.  The window [a, e) holds the line samples c0..c1
        // (positions kLineKeys*c in [a, e)); their lower bound i (c0..c1
        // + 1) leaves one candidate range: positions after sample i - 1
        // (which is < x) up to sample i (which is >= x), clipped to the
        // window, at most kLineKeys - 1 positions of one line of R.  A
        // found sample i at the range's end sets the found bit the way a
        // read of R there would.  The samples are a sixteenth of R (one
        // per 128-byte line), so the first stage's reads stay in a
        // smaller, better-cached array and one line of R is read per
        // key.
        // (The direct probe on an index with short windows searches R in
        // one stage, which takes fewer steps there.)
        if (kTwoStage && two_stage) {
            uint32_t a[kItems], e[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                a[k] = first[k];
                e[k] = first[k] + len[k];
                const uint32_t c0 = (a[k] + kLineKeys - 1) / kLineKeys;
                const uint32_t c1 = len[k] ? (e[k] - 1) / kLineKeys : 0u;
                const bool some = len[k] != 0 && c1 >= c0;
                first[k] = c0;
                len[k] = some ? c1 - c0 + 1 : 0u;
            }
            bisect_lockstep<kItems>(RS, x, first, len, eqmask);
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const uint32_t i = first[k];
                const uint32_t c0 = (a[k] + kLineKeys - 1) / kLineKeys;
                const bool past = e[k] <= i * kLineKeys;  // no sample >= x in the window
                const uint32_t lo = i == c0 ? a[k] : i * kLineKeys - (kLineKeys - 1);
                const uint32_t hi = past ? e[k] : i * kLineKeys;
                eqmask &= ~((past ? 1u : 0u) << k);
                first[k] = lo;
                len[k] = e[k] > a[k] ? hi - lo : 0u;
            }
        }
        bisect_lockstep<kItems>(R, x, first, len, eqmask);
    }

    // 4: run lengths.
#pragma unroll
    for (int k = 0; k < kItems; ++k) c[k] = (eqmask >> k) & 1u;
    if constexpr (!kUnique) {
        // Forward scan of equal keys, four positions at a time, bounded by
        // the window; kSetupChunk keys per pass to bound register use.  The
        // lines read here are the ones the search just touched.
#pragma unroll
        for (int k0 = 0; k0 < kItems; k0 += kSetupChunk) {
            uint32_t cur[kSetupChunk];
            bool act[kSetupChunk];
#pragma unroll
            for (int u = 0; u < kSetupChunk; ++u) {
                cur[u] = first[k0 + u] + 1;
                act[u] = c[k0 + u] && cur[u] < end[k0 + u];
            }
            for (;;) {
                bool any = false;
#pragma unroll
                for (int u = 0; u < kSetupChunk; ++u) any |= act[u];
                if (!any) break;
                uint64_t v[kSetupChunk][4];
#pragma unroll
                for (int u = 0; u < kSetupChunk; ++u)
#pragma unroll
                    for (int w4 = 0; w4 < 4; ++w4) {
                        const bool in = act[u] && cur[u] + w4 < end[k0 + u];
                        v[u][w4] = R[in ? cur[u] + w4 : 0];
                        if (!in) v[u][w4] = ~x[k0 + u];
                    }
#pragma unroll
                for (int u = 0; u < kSetupChunk; ++u) {
                    bool run = act[u];
#pragma unroll
                    for (int w4 = 0; w4 < 4; ++w4) {
                        run = run && v[u][w4] == x[k0 + u];
                        c[k0 + u] += run ? 1u : 0u;
                    }
                    cur[u] += 4;
                    act[u] = run && cur[u] < end[k0 + u];
                }
            }
        }
    }
}

// Slots are read as whole 16-byte vectors: key, payload and gap flag.
__device__ inline uint4 load_slot(const GSlot* p) { return *(const uint4*)p; }
__device__ inline uint64_t slot_key(const uint4& v) {
    return (uint64_t)v.x | ((uint64_t)v.y << 32);
}

// Steps 1-3 on a gapped index (Section III-A, "GRMI Lookup") for the keys
// of one tile (layout as in search_keys): root model, leaf model, predicted
// slot sp, and the search state of each key: the slots [a, b) not yet known
// to hold a smaller key, starting as [sp, sp + the leaf's largest insertion
// drift] (empty for an empty leaf or a key past the end of s), and the
// gallop step.
template <class Leaf, int kItems>
__device__ __forceinline__ void gapped_setup(const uint32_t nslots, const uint32_t G,
                                             const Leaf* leaves, const RootModel& root,
                                             const uint32_t* rtab,
                                             const uint64_t* s, const uint64_t m,
                                             const uint64_t tbase, const uint32_t kpl,
                                             uint64_t (&x)[kItems], uint32_t (&a)[kItems],
                                             uint32_t (&b)[kItems], uint32_t (&step)[kItems]) {
    const int tid = threadIdx.x;
    uint32_t validmask = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = tbase + (uint64_t)k * kBlock + tid;
        const bool ok = (uint32_t)k < kpl && q < m;
        validmask |= (ok ? 1u : 0u) << k;
        x[k] = s[ok ? q : m - 1];
    }
#pragma unroll
    for (int k0 = 0; k0 < kItems; k0 += kSetupChunk) {
        Leaf lf[kSetupChunk];
#pragma unroll
        for (int u = 0; u < kSetupChunk; ++u)
            lf[u] = load_leaf(leaves + route_lds(root, rtab, x[k0 + u]));
#pragma unroll
        for (int u = 0; u < kSetupChunk; ++u) {
            const int k = k0 + u;
            const bool live = ((validmask >> k) & 1u) && lf[u].cnt != 0;
            const uint64_t sp = live ? gapped_pred(lf[u], x[k], G) : 0;
            uint64_t e = sp + (uint64_t)(lf[u].hi < 0 ? 0 : lf[u].hi);
            if (e > (uint64_t)nslots - 1) e = (uint64_t)nslots - 1;
            a[k] = live ? (uint32_t)sp : 0;
            b[k] = live ? (uint32_t)e + 1 : 0;
            step[k] = 1;
        }
    }
}

// Up to kMaxSteps lockstep search steps of the gapped lookup for the keys of
// a lane: each step probes one slot per unfinished key, galloping (slots
// a, a + 1, a + 3, a + 7, ... relative to the last slot known to hold a
// smaller key) until a slot holds a key >= x, then bisecting that bracket.
// A key is done when a == b; b is then its lower bound in the slots from
// sp on, bit k of eqmask says whether that slot is a key slot holding x,
// and first[k] is its payload.
template <int kItems, uint32_t kMaxSteps = 0>  // 0: until every key is done
__device__ __forceinline__ void gapped_steps(const GSlot* __restrict__ slots,
                                             const uint64_t (&x)[kItems],
                                             uint32_t (&a)[kItems], uint32_t (&b)[kItems],
                                             uint32_t (&step)[kItems], uint32_t& eqmask,
                                             uint32_t (&first)[kItems]) {
    static_assert(kItems <= 32, "eqmask holds one bit per key");
    for (uint32_t it = 0; kMaxSteps == 0 || it < kMaxSteps; ++it) {
        uint32_t any = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) any |= a[k] < b[k] ? 1u : 0u;
        if (!any) break;
        uint4 v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t g = a[k] - 1 + step[k];
            const uint32_t p = step[k] ? (g < b[k] - 1 ? g : b[k] - 1) : a[k] + ((b[k] - a[k]) >> 1);
            v[k] = load_slot(slots + (a[k] < b[k] ? p : 0u));
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t g = a[k] - 1 + step[k];
            const uint32_t p = step[k] ? (g < b[k] - 1 ? g : b[k] - 1) : a[k] + ((b[k] - a[k]) >> 1);
            const uint32_t act = a[k] < b[k] ? 1u : 0u;
            const uint64_t key = slot_key(v[k]);
            const uint32_t lt = key < x[k] ? act : 0u;
            const uint32_t ge = act ^ lt;
            // A trailing gap holds UINT64_MAX: only a key slot is a match.
            const uint32_t eq = key == x[k] && v[k].z != kGap ? 1u : 0u;
            a[k] = lt ? p + 1 : a[k];
            b[k] = ge ? p : b[k];
            step[k] = lt ? step[k] * 2 : (ge ? 0u : step[k]);
            eqmask = (eqmask & ~(ge << k)) | ((eq & ge) << k);
            first[k] = ge ? v[k].z : first[k];
        }
    }
}

// Steps 1-4 on a gapped index for the keys of one tile: setup, the search
// to the end, and (duplicates) the length of the match run.  The lower
// bound found is the slot of the first copy of x when x is in R (every slot
// between sp and it holds a smaller key), so its payload is the position of
// that copy; copies fill the next slots.  On return first[k] is that
// position and c[k] the number of copies (0 for a miss).
template <class Leaf, bool kUnique, int kItems>
__device__ __forceinline__ void search_keys_gapped(const GSlot* __restrict__ slots,
                                                   const uint32_t nslots, const uint32_t G,
                                                   const Leaf* leaves, const RootModel& root,
                                                   const uint32_t* rtab,
                                                   const uint64_t* s, const uint64_t m,
                                                   const uint64_t tbase, const uint32_t kpl,
                                                   uint32_t (&first)[kItems],
                                                   uint32_t (&c)[kItems]) {
    uint64_t x[kItems];
    uint32_t a[kItems], b[kItems], step[kItems];
    uint32_t eqmask = 0;
    gapped_setup<Leaf, kItems>(nslots, G, leaves, root, rtab, s, m, tbase, kpl, x, a, b, step);
#pragma unroll
    for (int k = 0; k < kItems; ++k) first[k] = 0;
    gapped_steps<kItems>(slots, x, a, b, step, eqmask, first);
#pragma unroll
    for (int k = 0; k < kItems; ++k) c[k] = (eqmask >> k) & 1u;
    if constexpr (!kUnique) {
        // Copies of x sit in the slots after b: count them, four at a time.
        uint32_t cur[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) cur[k] = b[k] + 1;
#pragma unroll
        for (int k0 = 0; k0 < kItems; k0 += kSetupChunk) {
            bool act[kSetupChunk];
#pragma unroll
            for (int u = 0; u < kSetupChunk; ++u)
                act[u] = c[k0 + u] && cur[k0 + u] < nslots;
            for (;;) {
                bool anyact = false;
#pragma unroll
                for (int u = 0; u < kSetupChunk; ++u) anyact |= act[u];
                if (!anyact) break;
                uint4 v[kSetupChunk][4];
#pragma unroll
                for (int u = 0; u < kSetupChunk; ++u)
#pragma unroll
                    for (int w4 = 0; w4 < 4; ++w4) {
                        const bool in = act[u] && cur[k0 + u] + w4 < nslots;
                        v[u][w4] = load_slot(slots + (in ? cur[k0 + u] + w4 : 0u));
                        if (!in) v[u][w4].x = ~(uint32_t)x[k0 + u];  // not equal to x
                    }
#pragma unroll
                for (int u = 0; u < kSetupChunk; ++u) {
                    bool run = act[u];
#pragma unroll
                    for (int w4 = 0; w4 < 4; ++w4) {
                        run = run && slot_key(v[u][w4]) == x[k0 + u] && v[u][w4].z != kGap;
                        c[k0 + u] += run ? 1u : 0u;
                    }
                    cur[k0 + u] += 4;
                    act[u] = run && cur[k0 + u] < nslots;
                }
            }
        }
    }
}

// Steps 1-4 on a learned hash index (Section III-C) for the keys of one
// tile (layout as in search_keys): root model, leaf model, bucket of the
// key, then a lockstep walk of each key's bucket chain, one 64-byte bucket
// per step, counting the slots that hold x.  Keys of R sit in their chain
// in R order, so the first match is the first copy of x.  A key stops at
// its first match when R has no duplicates, else at the end of its chain.
template <class Leaf, bool kUnique, int kItems>
__device__ __forceinline__ void search_keys_hash(const HBucket* __restrict__ buckets,
                                                 const uint32_t spk, const Leaf* leaves,
                                                 const RootModel& root, const uint32_t* rtab,
                                                 const uint64_t* s,
                                                 const uint64_t m, const uint64_t tbase,
                                                 const uint32_t kpl, uint32_t (&first)[kItems],
                                                 uint32_t (&c)[kItems]) {
    const int tid = threadIdx.x;
    uint64_t x[kItems];
    uint32_t cur[kItems];  // bucket to read next, or kNoBucket
    uint32_t validmask = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = tbase + (uint64_t)k * kBlock + tid;
        const bool ok = (uint32_t)k < kpl && q < m;
        validmask |= (ok ? 1u : 0u) << k;
        x[k] = s[ok ? q : m - 1];
    }
#pragma unroll
    for (int k0 = 0; k0 < kItems; k0 += kSetupChunk) {
        Leaf lf[kSetupChunk];
#pragma unroll
        for (int u = 0; u < kSetupChunk; ++u)
            lf[u] = load_leaf(leaves + route_lds(root, rtab, x[k0 + u]));
#pragma unroll
        for (int u = 0; u < kSetupChunk; ++u) {
            const int k = k0 + u;
            const bool live = ((validmask >> k) & 1u) && lf[u].cnt != 0;
            cur[k] = live ? (uint32_t)hash_bucket(lf[u], x[k], spk) : kNoBucket;
            first[k] = 0;
            c[k] = 0;
        }
    }
    for (;;) {
        uint32_t any = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) any |= cur[k] != kNoBucket ? 1u : 0u;
        if (!any) break;
        uint4 v[kItems][4];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint4* p = (const uint4*)(buckets + (cur[k] != kNoBucket ? cur[k] : 0u));
#pragma unroll
            for (int w = 0; w < 4; ++w) v[k][w] = p[w];
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const bool act = cur[k] != kNoBucket;
            const uint32_t nk = v[k][3].y;
            const uint64_t key[4] = {(uint64_t)v[k][0].x | ((uint64_t)v[k][0].y << 32),
                                     (uint64_t)v[k][0].z | ((uint64_t)v[k][0].w << 32),
                                     (uint64_t)v[k][1].x | ((uint64_t)v[k][1].y << 32),
                                     (uint64_t)v[k][1].z | ((uint64_t)v[k][1].w << 32)};
            const uint32_t rid[4] = {v[k][2].x, v[k][2].y, v[k][2].z, v[k][2].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t hit = act && (uint32_t)j < nk && key[j] == x[k] ? 1u : 0u;
                first[k] = hit && c[k] == 0 ? rid[j] : first[k];
                c[k] += hit;
            }
            cur[k] = !act || (kUnique && c[k] != 0) ? kNoBucket : v[k][3].x;
        }
    }
}

// Steps 5-7 for one tile whose lower bounds and run lengths are known:
// offsets, look-back, pair emission; then the tile is counted as done.
template <bool kUnique, int kItems, bool kWithOffsets>
__device__ __forceinline__ void emit_tile(const TileJob& j, const uint32_t tile,
                                          const uint32_t kpl,
                                          TileShared<kItems, kWithOffsets>& sh,
                                          const uint32_t (&first)[kItems],
                                          const uint32_t (&c)[kItems]) {
    static_assert(kUnique || kWithOffsets, "the duplicate path needs LDS offsets");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const uint64_t tbase = (uint64_t)tile * kBlock * kpl;
    if constexpr (kUnique) {
        // 5: ballot/popcount offsets; key order in the tile is (k, wave, lane).
        uint32_t lane_off[kItems];
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            uint64_t mask = __ballot(c[k] != 0);
            lane_off[k] = (uint32_t)__popcll(mask & lt);
            if (lane == 0) sh.wsum[k * (kBlock / 64) + wave] = (uint64_t)__popcll(mask);
        }
        __syncthreads();
        uint64_t total = 0;
#pragma unroll
        for (int q = 0; q < kItems * (kBlock / 64); ++q) total += sh.wsum[q];
        // 6: look-back.
        if (wave == 0) {
            uint64_t e = look_back(j.status, tile, total, j.err, lane);
            if (lane == 0) sh.excl = e;
        }
        __syncthreads();
        const uint64_t excl = sh.excl;
        // 7: one store per match.
        if (j.out) {
            uint64_t pre = 0;
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                uint64_t wpre = 0;
                for (int w = 0; w < wave; ++w) wpre += sh.wsum[k * (kBlock / 64) + w];
                uint64_t pos = excl + pre + wpre + lane_off[k];
                if (c[k] && pos < j.cap) {
                    lj_pair pr;
                    pr.s_idx = (uint32_t)(tbase + (uint64_t)k * kBlock + tid);
                    pr.r_idx = first[k];
                    j.out[pos] = pr;
                }
#pragma unroll
                for (int w = 0; w < kBlock / 64; ++w) pre += sh.wsum[k * (kBlock / 64) + w];
            }
        }
    } else {
        // 5: LDS scan of the counts in tile order.
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            int q = k * kBlock + tid;
            sh.off[q] = c[k];
            sh.j0[q] = first[k];
        }
        __syncthreads();
        uint64_t loc[kItems];
        uint64_t tsum = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            loc[i] = tsum;
            tsum += sh.off[tid * kItems + i];
        }
        uint64_t incl = wave_incl_scan(tsum, lane);
        if (lane == 63) sh.wsum[wave] = incl;
        __syncthreads();
        uint64_t wpre = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            if (w < wave) wpre += sh.wsum[w];
            total += sh.wsum[w];
        }
        const uint64_t texcl = wpre + incl - tsum;
#pragma unroll
        for (int i = 0; i < kItems; ++i) sh.off[tid * kItems + i] = texcl + loc[i];
        if (tid == 0) sh.off[(kBlock * kItems)] = total;
        // 6: look-back.
        if (wave == 0) {
            uint64_t e = look_back(j.status, tile, total, j.err, lane);
            if (lane == 0) sh.excl = e;
        }
        __syncthreads();
        const uint64_t excl = sh.excl;
        // 7: load-balanced emission of the tile's outputs.
        if (j.out && excl < j.cap) {
            uint64_t limit = j.cap - excl < total ? j.cap - excl : total;
            for (uint64_t o = tid; o < limit; o += kBlock) {
                // last q with sh.off[q] <= o
                int lo = 0, hi = (kBlock * kItems);  // sh.off[(kBlock * kItems)] = total > o
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (sh.off[mid] <= o) lo = mid;
                    else hi = mid;
                }
                lj_pair pr;
                pr.s_idx = (uint32_t)(tbase + (uint64_t)lo);
                pr.r_idx = sh.j0[lo] + (uint32_t)(o - sh.off[lo]);
                j.out[excl + o] = pr;
            }
        }
    }
    __syncthreads();  // the block's LDS is reused by the next tile
    finish_tile(j);
}

// Last-mile search of a launch: binary or exponential search of R within
// the RMI window, or the gapped index's search.
constexpr int kSearchBinary = 0;
constexpr int kSearchExp = 1;
constexpr int kSearchGapped = 2;
constexpr int kSearchHash = 3;
constexpr int kSearchOneStage = 4;  // binary search of R without the line-sample stage

// Probe one tile of a batch (steps 1-7).
template <class Leaf, bool kUnique, int kItems, bool kWithOffsets, int kSearch>
__device__ __forceinline__ void probe_tile(const TileJob& j, const uint32_t* rtab,
                                           const uint32_t tile, const uint32_t kpl,
                                           TileShared<kItems, kWithOffsets>& sh) {
    uint32_t first[kItems], c[kItems];
    if constexpr (kSearch == kSearchHash)
        search_keys_hash<Leaf, kUnique, kItems>(j.buckets, j.hash_spk, (const Leaf*)j.leaves,
                                                j.root, rtab, j.s, j.m,
                                                (uint64_t)tile * kBlock * kpl, kpl, first, c);
    else if constexpr (kSearch == kSearchGapped)
        search_keys_gapped<Leaf, kUnique, kItems>(j.slots, j.nslots, j.gap,
                                                  (const Leaf*)j.leaves, j.root, rtab, j.s, j.m,
                                                  (uint64_t)tile * kBlock * kpl, kpl, first, c);
    else
        search_keys<Leaf, kUnique, kItems, kSearch == kSearchExp, kSearch != kSearchOneStage>(
            j.r, j.rs, (const Leaf*)j.leaves, j.root, rtab, j.s, j.m,
            (uint64_t)tile * kBlock * kpl, kpl, first, c);
    emit_tile<kUnique, kItems, kWithOffsets>(j, tile, kpl, sh, first, c);
}

template <class Leaf, bool kUnique, int kItems, int kSearch>
__device__ __forceinline__ void probe_join_body(const TileJob& j, uint32_t* tile_counter) {
    __shared__ uint32_t s_tile;
    __shared__ TileShared<kItems, !kUnique> sh;
    __shared__ __align__(16) uint32_t s_root[kRootTabLen];
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
    stage_root(j.root, s_root);
    __syncthreads();
    probe_tile<Leaf, kUnique, kItems, !kUnique, kSearch>(j, s_root, s_tile, kItems, sh);
}

// The direct probe on a plain RMI without duplicate keys (binary or
// exponential search of R) runs at most two waves per SIMD: its keys miss
// every cache, and with more resident waves the extra misses in flight only
// queue and evict each other's lines (measured on lognormal-zipf-200M: two
// or three waves are 5-6% faster than the five its registers allow, and two
// read 1.90 L2->HBM lines per key against 2.16 with three, at the same
// speed).  probe_join_full_kernel keeps the full occupancy for the
// duplicate-key probe (4 keys per lane: it needs every wave's loads in
// flight; two waves cost it 17%) and for the gapped and hash searches.
template <class Leaf, bool kUnique, int kItems, int kSearch>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void
probe_join_kernel(TileJob j, uint32_t* tile_counter) {
    probe_join_body<Leaf, kUnique, kItems, kSearch>(j, tile_counter);
}
template <class Leaf, bool kUnique, int kItems, int kSearch>
__global__ __launch_bounds__(kBlock) void probe_join_full_kernel(TileJob j,
                                                                 uint32_t* tile_counter) {
    probe_join_body<Leaf, kUnique, kItems, kSearch>(j, tile_counter);
}

// Search kernel of the binned probe: keys in bin order, tiles of kBlock *
// kItems keys; the tiles are split into kXcds contiguous ranges and
// workgroup g works on range g % kXcds, so that each XCD's L2 holds the R
// lines of its own few key ranges.  res[q] = lower bound of keys[q] when
// found, else ~0u (unique R); res[q] = lower bound | count << 32, or 0
// (duplicates).  A gapped index passes its slots, slot count and slots per
// key as well.
template <class Leaf, bool kUnique, int kItems, int kSearch>
__global__ __launch_bounds__(kBlock) void probe_binned_kernel(
    const uint64_t* __restrict__ R, const uint64_t* __restrict__ RS, const Leaf* leaves,
    RootModel root, const GSlot* __restrict__ slots, uint32_t nslots, uint32_t G,
    const HBucket* __restrict__ buckets, uint32_t hash_spk, const uint64_t* keys,
    uint64_t m, uint32_t ntiles, uint32_t tiles_per_xcd, void* res) {
    const uint32_t slot = blockIdx.x / kXcds;
    const uint32_t tile = (blockIdx.x % kXcds) * tiles_per_xcd + slot;
    if (slot >= tiles_per_xcd || tile >= ntiles) return;
    __shared__ __align__(16) uint32_t s_root[kRootTabLen];
    stage_root(root, s_root);
    __syncthreads();
    const uint64_t tbase = (uint64_t)tile * kBlock * kItems;
    uint32_t first[kItems], c[kItems];
    if constexpr (kSearch == kSearchHash)
        search_keys_hash<Leaf, kUnique, kItems>(buckets, hash_spk, leaves, root, s_root, keys, m,
                                                tbase, kItems, first, c);
    else if constexpr (kSearch == kSearchGapped)
        search_keys_gapped<Leaf, kUnique, kItems>(slots, nslots, G, leaves, root, s_root, keys, m,
                                                  tbase, kItems, first, c);
    else
        search_keys<Leaf, kUnique, kItems, kSearch == kSearchExp>(R, RS, leaves, root, s_root,
                                                                  keys, m, tbase, kItems, first,
                                                                  c);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = tbase + (uint64_t)k * kBlock + threadIdx.x;
        if (q >= m) continue;
        if constexpr (kUnique) ((uint32_t*)res)[q] = c[k] ? first[k] : ~0u;
        else ((uint64_t*)res)[q] = c[k] ? (uint64_t)first[k] | ((uint64_t)c[k] << 32) : 0ull;
    }
}

// Search kernels of the binned probe on a gapped index without duplicate
// keys.  Most keys sit at their predicted slot or a few slots after it, a
// few far away; a lockstep search over a tile runs as long as its slowest
// key, so the search is split.  First pass: every key gets kFirstSteps
// lockstep steps; a key that is then done writes its result (layout of
// probe_binned_kernel), the others go to a queue as (position in keys,
// a, b).  Second pass (gapped_queue_kernel): the queued keys, now dense,
// bisect their remaining slot range [a, b).  A wave whose keys do not fit
// in the queue finishes them in the first pass and marks any queue entries
// it took as void.
template <class Leaf, int kItems, uint32_t kFirstSteps>
__global__ __launch_bounds__(kBlock) void probe_binned_gapped_kernel(
    const Leaf* leaves, RootModel root, const GSlot* __restrict__ slots, uint32_t nslots,
    uint32_t G, const uint64_t* keys, uint64_t m, uint32_t ntiles, uint32_t tiles_per_xcd,
    uint32_t* res, uint4* queue, uint32_t qcap, uint32_t* qcount) {
    const uint32_t wslot = blockIdx.x / kXcds;
    const uint32_t tile = (blockIdx.x % kXcds) * tiles_per_xcd + wslot;
    if (wslot >= tiles_per_xcd || tile >= ntiles) return;
    __shared__ __align__(16) uint32_t s_root[kRootTabLen];
    stage_root(root, s_root);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t tbase = (uint64_t)tile * kBlock * kItems;
    uint64_t x[kItems];
    uint32_t a[kItems], b[kItems], step[kItems], first[kItems];
    uint32_t eqmask = 0;
    gapped_setup<Leaf, kItems>(nslots, G, leaves, root, s_root, keys, m, tbase, kItems, x, a, b,
                               step);
#pragma unroll
    for (int k = 0; k < kItems; ++k) first[k] = 0;
    gapped_steps<kItems, kFirstSteps>(slots, x, a, b, step, eqmask, first);

    // Reserve queue entries for the wave's unfinished keys.
    uint32_t open = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool u = a[k] < b[k];
        open |= (u ? 1u : 0u) << k;
        total += (uint32_t)__popcll(__ballot(u));
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (total) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(qcount, total);
        base = (uint32_t)__shfl((int)base, 0, 64);
        const bool fits = (uint64_t)base + total <= qcap;
        uint32_t off = base;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const bool u = (open >> k) & 1u;
            const uint64_t mask = __ballot(u);
            const uint32_t e = off + (uint32_t)__popcll(mask & lt);
            if (u && e < qcap) {
                const uint32_t q = (uint32_t)(tbase + (uint64_t)k * kBlock + threadIdx.x);
                queue[e] = fits ? make_uint4(q, a[k], b[k], 0u) : make_uint4(~0u, 0u, 0u, 0u);
            }
            off += (uint32_t)__popcll(mask);
        }
        if (!fits) {  // the whole wave finishes here (a wave-uniform branch)
            gapped_steps<kItems>(slots, x, a, b, step, eqmask, first);
            open = 0;
        }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = tbase + (uint64_t)k * kBlock + threadIdx.x;
        if (q < m && !((open >> k) & 1u)) res[q] = ((eqmask >> k) & 1u) ? first[k] : ~0u;
    }
}

// Second pass of the gapped search: queued keys in tiles of kBlock * kItems
// entries, dealt to the workgroups in turn.  Each key bisects [a, b); its
// lower bound b is then a slot holding a key >= x, or the end of its slot
// window, so the key slot of x is at b when x is in R (R has no duplicate
// keys: x occupies one slot, inside the window).
template <int kItems>
__global__ __launch_bounds__(kBlock) void gapped_queue_kernel(const GSlot* __restrict__ slots,
                                                              uint32_t nslots,
                                                              const uint64_t* keys,
                                                              const uint4* queue, uint32_t qcap,
                                                              const uint32_t* qcount,
                                                              uint32_t* res) {
    const uint32_t n = *qcount < qcap ? *qcount : qcap;
    const uint32_t per_tile = kBlock * kItems;
    for (uint32_t t0 = blockIdx.x * per_tile; t0 < n; t0 += gridDim.x * per_tile) {
        uint32_t q[kItems], a[kItems], b[kItems];
        uint64_t x[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t e = t0 + (uint32_t)k * kBlock + threadIdx.x;
            const uint4 v = e < n ? queue[e] : make_uint4(~0u, 0u, 0u, 0u);
            q[k] = v.x;
            a[k] = v.y;
            b[k] = v.z;
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) x[k] = q[k] != ~0u ? keys[q[k]] : 0ull;
        for (;;) {
            uint32_t any = 0;
#pragma unroll
            for (int k = 0; k < kItems; ++k) any |= a[k] < b[k] ? 1u : 0u;
            if (!any) break;
            uint4 v[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k)
                v[k] = load_slot(slots + (a[k] < b[k] ? a[k] + ((b[k] - a[k]) >> 1) : 0u));
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const uint32_t p = a[k] + ((b[k] - a[k]) >> 1);
                const bool act = a[k] < b[k];
                const bool lt = slot_key(v[k]) < x[k];
                a[k] = act && lt ? p + 1 : a[k];
                b[k] = act && !lt ? p : b[k];
            }
        }
        uint4 v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            v[k] = load_slot(slots + (q[k] != ~0u && b[k] < nslots ? b[k] : 0u));
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (q[k] == ~0u) continue;
            const bool hit = b[k] < nslots && slot_key(v[k]) == x[k] && v[k].z != kGap;
            res[q[k]] = hit ? v[k].z : ~0u;
        }
    }
}

// Last stage of the binned probe: puts the per-key results back in S order
// and emits the pairs in one pass.  res holds the results in pass-1 order
// (layout of probe_binned_kernel after the pass-2 gather); key p of S reads
// res[dest[p]], where dest[p] is its pass-1 position.  Tiles of kBlock *
// kItems keys of S, tile ids from an atomic counter, output offsets by
// decoupled look-back over the tiles -> steps 5-7 of the probe without
// writing the S-order results out and reading them back.  The tiles are
// larger than a partition chunk because every tile costs two updates of
// single counters, which the device serialises.
template <bool kUnique, int kItems>
__global__ __launch_bounds__(kBlock) void restore_emit_kernel(TileJob j,
                                                              const uint32_t* __restrict__ dest,
                                                              const void* __restrict__ res,
                                                              uint32_t* tile_counter) {
    __shared__ uint32_t s_tile;
    __shared__ TileShared<kItems, !kUnique> sh;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t tbase = (uint64_t)tile * kBlock * kItems;
    uint32_t first[kItems], c[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t q = tbase + (uint64_t)k * kBlock + threadIdx.x;
        first[k] = q < j.m ? dest[q] : ~0u;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t d = first[k];
        if constexpr (kUnique) {
            const uint32_t v = d != ~0u ? ((const uint32_t*)res)[d] : ~0u;
            first[k] = v;
            c[k] = v != ~0u ? 1u : 0u;
        } else {
            const uint64_t v = d != ~0u ? ((const uint64_t*)res)[d] : 0ull;
            first[k] = (uint32_t)v;
            c[k] = (uint32_t)(v >> 32);
        }
    }
    emit_tile<kUnique, kItems, !kUnique>(j, tile, kItems, sh, first, c);
}
constexpr int kItemsRestore = 32;     // unique R
constexpr int kItemsRestoreDup = 16;  // duplicates: LDS offsets per key

__global__ void zero_words(uint64_t* w, uint64_t nwords) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (uint64_t)gridDim.x * blockDim.x)
        w[i] = 0;
}

__global__ void line_samples_kernel(const uint64_t* __restrict__ r, uint64_t ns,
                                    uint64_t* __restrict__ rs) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns;
         i += (uint64_t)gridDim.x * blockDim.x)
        rs[i] = r[i * kLineKeys];
}

__global__ void set_u64_kernel(uint64_t* p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <class Leaf>
__global__ void self_check_kernel(const uint64_t* R, uint64_t n, const Leaf* leaves,
                                  RootModel root, unsigned long long* viol) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t x = R[i];
        const Leaf lf = leaves[route(root, x)];
        bool ok = lf.cnt != 0 && i >= lf.pos0 && i < (uint64_t)lf.pos0 + lf.cnt;
        if (ok) {
            int64_t e = (int64_t)(i - lf.pos0) - predict_rel(lf, x);
            ok = e >= lf.lo && e <= lf.hi;
        }
        if (!ok) atomicAdd(viol, 1ull);
    }
}

// Gapped index: every key slot must hold R at its payload position and sit
// inside its slot window; key slots are counted into nkeys.
template <class Leaf>
__global__ void self_check_gapped_kernel(const uint64_t* R, uint64_t n, const GSlot* slots,
                                         uint64_t nslots, uint32_t G, const Leaf* leaves,
                                         RootModel root, unsigned long long* viol,
                                         unsigned long long* nkeys) {
    uint32_t bad = 0, keys = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nslots;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = load_slot(slots + j);
        if (v.z == kGap) continue;
        ++keys;
        const uint64_t x = slot_key(v);
        const Leaf lf = leaves[route(root, x)];
        bool ok = v.z < n && R[v.z] == x && lf.cnt != 0 && v.z >= lf.pos0 &&
                  v.z < (uint64_t)lf.pos0 + lf.cnt;
        if (ok) {
            const uint64_t sp = gapped_pred(lf, x, G);
            ok = j >= sp && j - sp <= (uint64_t)(lf.hi < 0 ? 0 : lf.hi);
        }
        bad += ok ? 0u : 1u;
    }
    if (bad) atomicAdd(viol, (unsigned long long)bad);
    if (keys) atomicAdd(nkeys, (unsigned long long)keys);
}

// Learned hash index: every key of R must be found, with its own position,
// in the chain of its bucket (a chain longer than nbuckets is a violation,
// not a hang); bucket_keys_kernel counts the keys the buckets hold.
template <class Leaf>
__global__ void self_check_hash_kernel(const uint64_t* R, uint64_t n, const HBucket* buckets,
                                       uint64_t nbuckets, uint32_t spk, const Leaf* leaves,
                                       RootModel root, unsigned long long* viol) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = R[i];
        const Leaf lf = leaves[route(root, x)];
        bool found = false;
        if (lf.cnt != 0) {
            uint64_t b = hash_bucket(lf, x, spk);
            for (uint64_t hops = 0; b < nbuckets && hops < nbuckets && !found; ++hops) {
                const HBucket& h = buckets[b];
                for (uint32_t j = 0; j < kBucketSlots && j < h.nkeys; ++j)
                    found = found || (h.ridx[j] == (uint32_t)i && h.key[j] == x);
                b = h.next;
            }
        }
        bad += found ? 0u : 1u;
    }
    if (bad) atomicAdd(viol, (unsigned long long)bad);
}

__global__ void bucket_keys_kernel(const HBucket* buckets, uint64_t nbuckets,
                                   unsigned long long* nkeys) {
    uint32_t keys = 0;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nbuckets;
         b += (uint64_t)gridDim.x * blockDim.x)
        keys += buckets[b].nkeys;
    if (keys) atomicAdd(nkeys, (unsigned long long)keys);
}

// viol[0] += |nkeys - n|.
__global__ void finish_gapped_check_kernel(unsigned long long* viol, const unsigned long long* nkeys,
                                           uint64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        viol[0] += *nkeys > n ? *nkeys - n : n - *nkeys;
}

template <class Leaf>
__global__ void predict_windows_kernel(const uint64_t* keys, uint64_t m, const Leaf* leaves,
                                       RootModel root, uint32_t G, uint64_t nslots,
                                       uint32_t hash_spk, uint32_t* leaf_out, int64_t* pred,
                                       int64_t* wlo, int64_t* whi) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t x = keys[i];
        uint32_t l = route(root, x);
        const Leaf lf = leaves[l];
        int64_t lo = 1, hi = 0, pr = -1;
        if (lf.cnt != 0 && hash_spk) {
            pr = (int64_t)hash_bucket(lf, x, hash_spk);
            lo = hi = pr;
        } else if (lf.cnt != 0 && G) {
            pr = (int64_t)gapped_pred(lf, x, G);
            lo = pr;
            hi = pr + (lf.hi < 0 ? 0 : lf.hi);
            if (hi > (int64_t)nslots - 1) hi = (int64_t)nslots - 1;
        } else if (lf.cnt != 0) {
            int64_t rel = predict_rel(lf, x);
            pr = (int64_t)lf.pos0 + rel;
            int64_t a = rel + lf.lo, b = rel + lf.hi;
            if (a < 0) a = 0;
            if (b > (int64_t)lf.cnt - 1) b = (int64_t)lf.cnt - 1;
            if (a <= b) {
                lo = (int64_t)lf.pos0 + a;
                hi = (int64_t)lf.pos0 + b;
            }
        }
        if (leaf_out) leaf_out[i] = l;
        if (pred) pred[i] = pr;
        if (wlo) wlo[i] = lo;
        if (whi) whi[i] = hi;
    }
}

// Fused launch of many batches (one kernel for all the batches of a plan or
// of a serving batch).  Tiles of all batches share one id space: batch b
// owns ids [tile0_b, tile0_b + ntiles_b), its tiles in key order, and each
// thread block takes the next id from the launch's counter, so the
// look-back of a batch's tile only waits on tiles already handed to running
// blocks (which publish their aggregates before they wait on anything).
// The grid holds one block per tile: as blocks retire the dispatcher starts
// new ones, which keeps every CU's slots filled the way a loop over tile
// ids in long-lived blocks would; such a loop was tried and costs
// registers (the compiler keeps loop-invariant constants of the tile shapes
// live across iterations: 248-256 VGPRs, one wave per SIMD on unique R with
// tiles of up to 16 keys per lane, against 183 and two waves here).  A tile
// runs steps 1-7 of probe_tile with its batch's own keys per lane (4 or 8)
// and line-sample stage, using the LDS of the largest tile shape.
template <class Leaf, bool kUnique, int kItems, int kMaxItems, int kSearch>
__device__ __forceinline__ void fused_tile(const TileJob& j, const uint32_t* rtab,
                                           const uint32_t tile, const bool two_stage,
                                           char* lds) {
    using Sh = TileShared<kItems, !kUnique>;
    static_assert(sizeof(Sh) <= sizeof(TileShared<kMaxItems, !kUnique>), "LDS of a tile");
    Sh& sh = *reinterpret_cast<Sh*>(lds);
    uint32_t first[kItems], c[kItems];
    const uint64_t tbase = (uint64_t)tile * kBlock * kItems;
    if constexpr (kSearch == kSearchGapped)
        search_keys_gapped<Leaf, kUnique, kItems>(j.slots, j.nslots, j.gap,
                                                  (const Leaf*)j.leaves, j.root, rtab, j.s, j.m,
                                                  tbase, kItems, first, c);
    else
        search_keys<Leaf, kUnique, kItems, false>(j.r, j.rs, (const Leaf*)j.leaves, j.root,
                                                  rtab, j.s, j.m, tbase, kItems, first, c,
                                                  two_stage);
    emit_tile<kUnique, kItems, !kUnique>(j, tile, kItems, sh, first, c);
}

// kSearch: kSearchBinary (plain RMI; each batch's own line-sample stage) or
// kSearchGapped (gapped RMI).  The kernel's registers are those of its
// largest tile shape, so it offers at most kItemsFused (kItemsGapped) keys
// per lane: deeper tiles would cut the waves per SIMD of every tile.
template <class Leaf, bool kUnique, int kSearch>
__device__ __forceinline__ void fused_body(const FusedJob* __restrict__ jobs, uint32_t njobs,
                                           uint32_t total_tiles, uint32_t* tile_counter) {
    constexpr int kMax = kSearch == kSearchGapped ? kItemsGapped : kItemsFused;
    __shared__ __align__(16) char lds[sizeof(TileShared<kMax, !kUnique>)];
    __shared__ __align__(16) uint32_t s_root[kRootTabLen];
    __shared__ uint32_t s_tile, s_job;
    if (threadIdx.x == 0) {
        const uint32_t t = atomicAdd(tile_counter, 1u);  // < total_tiles: one block per tile
        uint32_t lo = 0, hi = njobs;  // the last batch whose first tile id is <= t
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (jobs[mid].tile0 <= t) lo = mid;
            else hi = mid;
        }
        s_tile = t;
        s_job = lo;
    }
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_tile);
    const uint32_t b = __builtin_amdgcn_readfirstlane(s_job);
    if (t >= total_tiles) return;  // cannot happen: the grid has total_tiles blocks
    const TileJob& j = jobs[b].j;
    stage_root(j.root, s_root);
    __syncthreads();
    const uint32_t tile = t - jobs[b].tile0;
    const bool two = jobs[b].two_stage != 0;
    static_assert(kMax == 8 || kMax == 16, "fused tiles: 4, 8 or 16 keys per lane");
    if (j.kpl == 4) {
        fused_tile<Leaf, kUnique, 4, kMax, kSearch>(j, s_root, tile, two, lds);
    } else if constexpr (kMax == 16) {
        if (j.kpl == 8) fused_tile<Leaf, kUnique, 8, kMax, kSearch>(j, s_root, tile, two, lds);
        else fused_tile<Leaf, kUnique, 16, kMax, kSearch>(j, s_root, tile, two, lds);
    } else {
        fused_tile<Leaf, kUnique, 8, kMax, kSearch>(j, s_root, tile, two, lds);
    }
}

// Plain RMIs at most three waves per SIMD (a fused launch of many batches
// measured 2% faster with three than with two); gapped RMIs at full
// occupancy, as probe_join_full_kernel.
template <class Leaf, bool kUnique>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 3))) void
probe_fused_kernel(const FusedJob* __restrict__ jobs, uint32_t njobs, uint32_t total_tiles,
                   uint32_t* tile_counter) {
    fused_body<Leaf, kUnique, kSearchBinary>(jobs, njobs, total_tiles, tile_counter);
}
template <class Leaf, bool kUnique>
__global__ __launch_bounds__(kBlock) void probe_fused_gapped_kernel(
    const FusedJob* __restrict__ jobs, uint32_t njobs, uint32_t total_tiles,
    uint32_t* tile_counter) {
    fused_body<Leaf, kUnique, kSearchGapped>(jobs, njobs, total_tiles, tile_counter);
}

// Clears what a fused launch needs zeroed: the shared header (tile counter,
// error flag) and every batch's done counter and look-back status words.
// One block per batch; block 0 also clears the header.
__global__ void zero_fused_kernel(const FusedJob* __restrict__ jobs, uint32_t* hdr_words,
                                  uint32_t hdr_count) {
    const FusedJob& fj = jobs[blockIdx.x];
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < hdr_count; i += blockDim.x) hdr_words[i] = 0u;
    if (threadIdx.x == 0) *fj.j.done = 0u;
    for (uint32_t i = threadIdx.x; i < fj.j.ntiles; i += blockDim.x) fj.j.status[i] = 0ull;
}

unsigned grid_for(uint64_t work, unsigned block) {
    uint64_t g = (work + block - 1) / block;
    if (g > 65536) g = 65536;
    return (unsigned)(g ? g : 1);
}

}  // namespace

hipError_t launch_line_samples(const uint64_t* r, uint64_t n, uint64_t* rs,
                               hipStream_t stream) {
    const uint64_t ns = (n + kLineKeys - 1) / kLineKeys;
    if (ns == 0) return hipSuccess;
    hipLaunchKernelGGL(line_samples_kernel, dim3(grid_for(ns, 256)), dim3(256), 0, stream, r, ns,
                       rs);
    return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t* p, uint64_t v, hipStream_t stream) {
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, stream, p, v);
    return hipGetLastError();
}

hipError_t launch_zero_words(uint64_t* p, uint64_t nwords, hipStream_t stream) {
    hipLaunchKernelGGL(zero_words, dim3(grid_for(nwords, 256)), dim3(256), 0, stream, p, nwords);
    return hipGetLastError();
}

namespace {

template <class Leaf, bool kUnique, int kItems, int kSearch>
hipError_t launch_join(const TileJob& j, uint32_t* ctr, hipStream_t stream) {
    const dim3 grid(j.ntiles), block(kBlock);
    if constexpr (!kUnique || kSearch == kSearchGapped || kSearch == kSearchHash)
        hipLaunchKernelGGL((probe_join_full_kernel<Leaf, kUnique, kItems, kSearch>), grid,
                           block, 0, stream, j, ctr);
    else
        hipLaunchKernelGGL((probe_join_kernel<Leaf, kUnique, kItems, kSearch>), grid, block, 0,
                           stream, j, ctr);
    return hipGetLastError();
}

template <int kItems, int kSearch>
hipError_t launch_probe_items(const TileJob& j, uint32_t* ctr, hipStream_t stream) {
    if constexpr (kSearch == kSearchHash && kItems > kItemsHash) {
        return hipErrorInvalidValue;  // launch_probe caps keys per lane for hash indexes
    } else {
        switch (j.kind & (kJobFp64 | kJobDup)) {
            case 0: return launch_join<LeafF32, true, kItems, kSearch>(j, ctr, stream);
            case kJobDup:
                if constexpr (kItems <= kItemsDupMax)
                    return launch_join<LeafF32, false, kItems, kSearch>(j, ctr, stream);
                else
                    return hipErrorInvalidValue;
            case kJobFp64: return launch_join<LeafF64, true, kItems, kSearch>(j, ctr, stream);
            default:
                if constexpr (kItems <= kItemsDupMax)
                    return launch_join<LeafF64, false, kItems, kSearch>(j, ctr, stream);
                else
                    return hipErrorInvalidValue;
        }
    }
}

}  // namespace

bool probe_kpl_supported(uint32_t kpl, bool dup) {
    return kpl == 4 || kpl == 8 || kpl == 16 || (!dup && kpl == 24);
}

namespace {

// The index's fields of a TileJob.
TileJob index_job(const lj_index* idx) {
    TileJob j{};
    j.r = idx->r_dev;
    j.rs = idx->rs_dev;
    j.leaves = idx->leaf_dev;
    j.root = idx->root;
    j.kind = job_kind(idx);
    j.slots = idx->slots_dev;
    j.nslots = (uint32_t)idx->nslots;
    j.gap = idx->gap;
    j.buckets = idx->buckets_dev;
    j.hash_spk = idx->hash_spk;
    return j;
}

int search_mode(uint32_t kind) {
    return (kind & kJobHash)     ? kSearchHash
           : (kind & kJobGapped) ? kSearchGapped
           : (kind & kJobExp)    ? kSearchExp
                                 : kSearchBinary;
}

// The direct probe's binary search: two stages unless the index's windows
// are short.
int direct_search_mode(const lj_index* idx, uint32_t kind) {
    const int mode = search_mode(kind);
    return mode == kSearchBinary && idx->mean_window < kTwoStageMinWindow ? kSearchOneStage
                                                                           : mode;
}

template <class Leaf, bool kUnique, int kSearch>
void launch_binned_search(const lj_index* idx, const uint64_t* keys, uint64_t m, void* res,
                          hipStream_t stream) {
    // A hash probe holds a whole 64-byte bucket per key in registers.
    constexpr int kItems = kSearch == kSearchHash ? kItemsHash : kItemsBinned;
    const uint32_t nt = (uint32_t)num_tiles(m, (uint64_t)kBlock * kItems);
    const uint32_t per = (nt + kXcds - 1) / kXcds;
    hipLaunchKernelGGL((probe_binned_kernel<Leaf, kUnique, kItems, kSearch>), dim3(per * kXcds),
                       dim3(kBlock), 0, stream, idx->r_dev, idx->rs_dev,
                       (const Leaf*)idx->leaf_dev, idx->root, idx->slots_dev,
                       (uint32_t)idx->nslots, idx->gap, idx->buckets_dev, idx->hash_spk, keys,
                       m, nt, per, res);
}

// Steps of the first pass of the two-pass gapped search, and keys per lane
// of its second pass.
constexpr uint32_t kGappedFirstSteps = 3;
constexpr int kGappedFirstItems = 16;
constexpr int kGappedQueueItems = 8;

// Two-pass search of a gapped index without duplicate keys; the queue lives
// in the workspace's bin arrays, which the partition no longer needs.
template <class Leaf>
void launch_binned_gapped(const lj_index* idx, const uint64_t* keys, uint64_t m, void* res,
                          void* ws, const BinnedWs& L, hipStream_t stream) {
    constexpr int kItems = kGappedFirstItems;
    const uint32_t nt = (uint32_t)num_tiles(m, (uint64_t)kBlock * kItems);
    const uint32_t per = (nt + kXcds - 1) / kXcds;
    uint4* queue = (uint4*)((char*)ws + L.bins_s);
    const uint32_t qcap = (uint32_t)((L.p1 - L.bins_s) / sizeof(uint4));
    uint32_t* qcount = &((WsHeader*)ws)->queue_count;
    hipLaunchKernelGGL((probe_binned_gapped_kernel<Leaf, kItems, kGappedFirstSteps>),
                       dim3(per * kXcds), dim3(kBlock), 0, stream, (const Leaf*)idx->leaf_dev,
                       idx->root, idx->slots_dev, (uint32_t)idx->nslots, idx->gap, keys, m, nt,
                       per, (uint32_t*)res, queue, qcap, qcount);
    const uint32_t qt = (uint32_t)num_tiles(qcap, (uint64_t)kBlock * kGappedQueueItems);
    const uint32_t grid = qt < 2048u ? (qt ? qt : 1u) : 2048u;
    hipLaunchKernelGGL(gapped_queue_kernel<kGappedQueueItems>, dim3(grid), dim3(kBlock), 0,
                       stream, idx->slots_dev, (uint32_t)idx->nslots, keys,
                       (const uint4*)queue, qcap, (const uint32_t*)qcount, (uint32_t*)res);
}

template <class Leaf, bool kUnique>
void launch_binned_search_any(int search, const lj_index* idx, const uint64_t* keys,
                              uint64_t m, void* res, void* ws, const BinnedWs& L,
                              hipStream_t stream) {
    if (search == kSearchHash)
        launch_binned_search<Leaf, kUnique, kSearchHash>(idx, keys, m, res, stream);
    else if (search == kSearchGapped && kUnique)
        launch_binned_gapped<Leaf>(idx, keys, m, res, ws, L, stream);
    else if (search == kSearchGapped)
        launch_binned_search<Leaf, kUnique, kSearchGapped>(idx, keys, m, res, stream);
    else if (search == kSearchExp)
        launch_binned_search<Leaf, kUnique, kSearchExp>(idx, keys, m, res, stream);
    else
        launch_binned_search<Leaf, kUnique, kSearchBinary>(idx, keys, m, res, stream);
}

// Binned probe: partition S by key range, search in that order, put the
// per-key results back in S order, emit.
hipError_t launch_probe_binned(const lj_index* idx, const uint64_t* s, uint64_t m,
                               lj_pair* out, uint64_t cap, uint64_t* count_dev, void* ws,
                               hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
    const uint32_t kind = job_kind(idx);
    const bool dup = (kind & kJobDup) != 0;
    const BinnedWs L = binned_ws(m);
    char* w = (char*)ws;
    hipError_t e = launch_zero_words((uint64_t*)ws, L.ctrl_bytes / 8, stream);
    if (e != hipSuccess) return e;
    e = launch_partition(idx, s, m, ws, L, stream);
    if (e != hipSuccess) return e;
    // res2 (bin order) in p1, res1 (pass-1 order) in p2.
    void* res2 = w + L.p1;
    void* res1 = w + L.p2;
    const uint64_t* keys = (const uint64_t*)(w + L.p2);
    if (ev0) {
        e = hipEventRecord(ev0, stream);
        if (e != hipSuccess) return e;
    }
    const int search = search_mode(kind);
    const bool f64 = (kind & kJobFp64) != 0;
    if (!f64 && !dup)
        launch_binned_search_any<LeafF32, true>(search, idx, keys, m, res2, ws, L, stream);
    else if (!f64)
        launch_binned_search_any<LeafF32, false>(search, idx, keys, m, res2, ws, L, stream);
    else if (!dup)
        launch_binned_search_any<LeafF64, true>(search, idx, keys, m, res2, ws, L, stream);
    else
        launch_binned_search_any<LeafF64, false>(search, idx, keys, m, res2, ws, L, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) {
        e = hipEventRecord(ev1, stream);
        if (e != hipSuccess) return e;
    }
    e = launch_unpermute((const uint32_t*)(w + L.dest2), res2, res1, m, dup, stream);
    if (e != hipSuccess) return e;

    // Chunk ids, finished chunks and per-chunk look-back words live in the
    // zeroed control block.
    WsHeader* hdr = (WsHeader*)ws;
    uint32_t* ctr = (uint32_t*)(w + L.scan_ctr);
    TileJob j{};
    j.s = s;
    j.m = m;
    j.out = out;
    j.cap = out ? cap : 0;
    j.count_out = count_dev;
    j.status = (uint64_t*)(w + L.counts);  // nchunks + 1 words >= tiles
    j.done = ctr + 32;                     // a cache line apart from the tile counter
    j.err = &hdr->err;
    j.kind = kind;
    j.kpl = dup ? kItemsRestoreDup : kItemsRestore;
    j.ntiles = (uint32_t)num_tiles(m, (uint64_t)kBlock * j.kpl);
    if (dup)
        hipLaunchKernelGGL((restore_emit_kernel<false, kItemsRestoreDup>), dim3(j.ntiles),
                           dim3(kBlock), 0, stream, j, (const uint32_t*)(w + L.dest1),
                           (const void*)res1, ctr + 2);
    else
        hipLaunchKernelGGL((restore_emit_kernel<true, kItemsRestore>), dim3(j.ntiles),
                           dim3(kBlock), 0, stream, j, (const uint32_t*)(w + L.dest1),
                           (const void*)res1, ctr + 2);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_probe(const lj_index* idx, const uint64_t* s, uint64_t m, lj_pair* out,
                        uint64_t cap, uint64_t* count_dev, void* ws, hipStream_t stream,
                        hipEvent_t ev0, hipEvent_t ev1, uint32_t kpl, int mode) {
    if (uses_binned(idx, m, mode))
        return launch_probe_binned(idx, s, m, out, cap, count_dev, ws, stream, ev0, ev1);
    const uint32_t kind = job_kind(idx);
    if (kpl == 0)
        kpl = (kind & kJobHash)     ? kItemsHash
              : (kind & kJobDup)    ? kItemsDup
              : (kind & kJobGapped) ? kItemsGapped
                                    : kItemsUnique;
    if (!probe_kpl_supported(kpl, (kind & kJobDup) != 0)) return hipErrorInvalidValue;
    if ((kind & kJobHash) && kpl > (uint32_t)kItemsHash) kpl = kItemsHash;
    const uint64_t nt = num_tiles(m, (uint64_t)kBlock * kpl);
    const uint64_t words = (kWsHeaderBytes + nt * 8) / 8;
    hipError_t e = launch_zero_words((uint64_t*)ws, words, stream);
    if (e != hipSuccess) return e;

    WsHeader* hdr = (WsHeader*)ws;
    TileJob j = index_job(idx);
    j.s = s;
    j.m = m;
    j.out = out;
    j.cap = out ? cap : 0;
    j.count_out = count_dev;
    j.status = (uint64_t*)((char*)ws + kWsHeaderBytes);
    j.done = &hdr->done_counter;
    j.err = &hdr->err;
    j.ntiles = (uint32_t)nt;
    j.kind = kind;
    j.kpl = kpl;

    if (ev0) {
        e = hipEventRecord(ev0, stream);
        if (e != hipSuccess) return e;
    }
    uint32_t* ctr = &hdr->tile_counter;
    const int search = direct_search_mode(idx, kind);
#define LJ_ITEMS(K)                                                                      \
    e = search == kSearchHash       ? launch_probe_items<K, kSearchHash>(j, ctr, stream)   \
        : search == kSearchGapped   ? launch_probe_items<K, kSearchGapped>(j, ctr, stream) \
        : search == kSearchExp      ? launch_probe_items<K, kSearchExp>(j, ctr, stream)    \
        : search == kSearchOneStage ? launch_probe_items<K, kSearchOneStage>(j, ctr, stream) \
                                    : launch_probe_items<K, kSearchBinary>(j, ctr, stream)
    switch (kpl) {
        case 4: LJ_ITEMS(4); break;
        case 8: LJ_ITEMS(8); break;
        case 16: LJ_ITEMS(16); break;
        default: LJ_ITEMS(24); break;
    }
#undef LJ_ITEMS
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, stream);
    return e;
}

int fused_group(const lj_index* idx) {
    const uint32_t kind = job_kind(idx);
    if (kind & (kJobExp | kJobHash)) return -1;
    return (int)(kind & (kJobFp64 | kJobDup)) + ((kind & kJobGapped) ? kFusedGroupGapped : 0);
}

uint32_t fused_kpl(const lj_index* idx, uint32_t kpl) {
    if (kpl != 4 && kpl != 8 && kpl != 16 && kpl != 24) kpl = 8;
    const uint32_t cap = idx->gap ? (uint32_t)kItemsGapped : (uint32_t)kItemsFused;
    return kpl < cap ? kpl : cap;
}

FusedJob make_fused_job(const lj_index* idx, const uint64_t* s, uint64_t m, lj_pair* out,
                        uint64_t cap, uint64_t* count_out, void* job_ws, uint32_t kpl,
                        uint32_t* err, uint32_t tile0) {
    FusedJob f{};
    f.j = index_job(idx);
    f.j.s = s;
    f.j.m = m;
    f.j.out = out;
    f.j.cap = out ? cap : 0;
    f.j.count_out = count_out;
    f.j.done = (uint32_t*)job_ws;
    f.j.status = (uint64_t*)((char*)job_ws + kFusedJobHeader);
    f.j.err = err;
    f.j.kpl = fused_kpl(idx, kpl);
    f.j.ntiles = (uint32_t)num_tiles(m, (uint64_t)kBlock * f.j.kpl);
    f.tile0 = tile0;
    f.two_stage = direct_search_mode(idx, f.j.kind) == kSearchBinary ? 1u : 0u;
    return f;
}

namespace {

template <class Leaf, bool kUnique, int kSearch>
hipError_t launch_fused_typed(const FusedJob* jobs, uint32_t njobs, uint32_t total_tiles,
                              uint32_t* tile_counter, hipStream_t stream) {
    if constexpr (kSearch == kSearchGapped)
        hipLaunchKernelGGL((probe_fused_gapped_kernel<Leaf, kUnique>), dim3(total_tiles),
                           dim3(kBlock), 0, stream, jobs, njobs, total_tiles, tile_counter);
    else
        hipLaunchKernelGGL((probe_fused_kernel<Leaf, kUnique>), dim3(total_tiles),
                           dim3(kBlock), 0, stream, jobs, njobs, total_tiles, tile_counter);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_probe_fused(const FusedJob* jobs_dev, uint32_t njobs, uint32_t total_tiles,
                              int group, uint32_t* hdr, hipStream_t stream) {
    if (njobs == 0 || total_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_fused_kernel, dim3(njobs), dim3(256), 0, stream, jobs_dev, hdr,
                       (uint32_t)(kFusedHeader / 4));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* ctr = hdr;
    constexpr int kB = kSearchBinary, kG = kSearchGapped, kGg = kFusedGroupGapped;
    switch (group) {
        case 0:
            return launch_fused_typed<LeafF32, true, kB>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kJobDup:
            return launch_fused_typed<LeafF32, false, kB>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kJobFp64:
            return launch_fused_typed<LeafF64, true, kB>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kJobFp64 | kJobDup:
            return launch_fused_typed<LeafF64, false, kB>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kGg:
            return launch_fused_typed<LeafF32, true, kG>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kGg + kJobDup:
            return launch_fused_typed<LeafF32, false, kG>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kGg + kJobFp64:
            return launch_fused_typed<LeafF64, true, kG>(jobs_dev, njobs, total_tiles, ctr, stream);
        case kGg + (kJobFp64 | kJobDup):
            return launch_fused_typed<LeafF64, false, kG>(jobs_dev, njobs, total_tiles, ctr, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_self_check(const lj_index* idx, uint64_t* viol, hipStream_t stream) {
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, viol, (uint64_t)2);
    if (idx->hash_spk) {
        unsigned long long* v = (unsigned long long*)viol;
        const unsigned g = grid_for(idx->n, 256);
        if (idx->n && leaf_fp32(idx->flags))
            hipLaunchKernelGGL(self_check_hash_kernel<LeafF32>, dim3(g), dim3(256), 0, stream,
                               idx->r_dev, idx->n, idx->buckets_dev, idx->nbuckets,
                               idx->hash_spk, (const LeafF32*)idx->leaf_dev, idx->root, v);
        else if (idx->n)
            hipLaunchKernelGGL(self_check_hash_kernel<LeafF64>, dim3(g), dim3(256), 0, stream,
                               idx->r_dev, idx->n, idx->buckets_dev, idx->nbuckets,
                               idx->hash_spk, (const LeafF64*)idx->leaf_dev, idx->root, v);
        hipLaunchKernelGGL(bucket_keys_kernel, dim3(grid_for(idx->nbuckets, 256)), dim3(256), 0,
                           stream, idx->buckets_dev, idx->nbuckets, v + 1);
        hipLaunchKernelGGL(finish_gapped_check_kernel, dim3(1), dim3(64), 0, stream, v,
                           (const unsigned long long*)(v + 1), idx->n);
        return hipGetLastError();
    }
    if (idx->gap) {
        unsigned long long* v = (unsigned long long*)viol;
        const unsigned gs = grid_for(idx->nslots, 256);
        if (leaf_fp32(idx->flags))
            hipLaunchKernelGGL(self_check_gapped_kernel<LeafF32>, dim3(gs), dim3(256), 0, stream,
                               idx->r_dev, idx->n, idx->slots_dev, idx->nslots, idx->gap,
                               (const LeafF32*)idx->leaf_dev, idx->root, v, v + 1);
        else
            hipLaunchKernelGGL(self_check_gapped_kernel<LeafF64>, dim3(gs), dim3(256), 0, stream,
                               idx->r_dev, idx->n, idx->slots_dev, idx->nslots, idx->gap,
                               (const LeafF64*)idx->leaf_dev, idx->root, v, v + 1);
        hipLaunchKernelGGL(finish_gapped_check_kernel, dim3(1), dim3(64), 0, stream, v,
                           (const unsigned long long*)(v + 1), idx->n);
        return hipGetLastError();
    }
    unsigned g = grid_for(idx->n, 256);
    if (idx->n == 0) return hipGetLastError();
    if (leaf_fp32(idx->flags))
        hipLaunchKernelGGL(self_check_kernel<LeafF32>, dim3(g), dim3(256), 0, stream,
                           idx->r_dev, idx->n, (const LeafF32*)idx->leaf_dev, idx->root,
                           (unsigned long long*)viol);
    else
        hipLaunchKernelGGL(self_check_kernel<LeafF64>, dim3(g), dim3(256), 0, stream,
                           idx->r_dev, idx->n, (const LeafF64*)idx->leaf_dev, idx->root,
                           (unsigned long long*)viol);
    return hipGetLastError();
}

hipError_t launch_predict_windows(const lj_index* idx, const uint64_t* keys, uint64_t m,
                                  uint32_t* leaf, int64_t* pred, int64_t* wlo, int64_t* whi,
                                  hipStream_t stream) {
    if (m == 0) return hipSuccess;
    unsigned g = grid_for(m, 256);
    if (leaf_fp32(idx->flags))
        hipLaunchKernelGGL(predict_windows_kernel<LeafF32>, dim3(g), dim3(256), 0, stream,
                           keys, m, (const LeafF32*)idx->leaf_dev, idx->root, idx->gap,
                           idx->nslots, idx->hash_spk, leaf, pred, wlo, whi);
    else
        hipLaunchKernelGGL(predict_windows_kernel<LeafF64>, dim3(g), dim3(256), 0, stream,
                           keys, m, (const LeafF64*)idx->leaf_dev, idx->root, idx->gap,
                           idx->nslots, idx->hash_spk, leaf, pred, wlo, whi);
    return hipGetLastError();
}

}  // namespace lj
