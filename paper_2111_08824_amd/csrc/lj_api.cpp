// C ABI of the learned indexed nested loop join (declared in include/lj.h):
// argument checks, device memory of the index, the per-stream workspace
// cache and the synchronous count readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <unordered_map>

#include "lj_internal.h"
#include "lj_sortjoin.h"

namespace {

constexpr uint64_t kMaxN = 1ull << 31;
constexpr uint64_t kMaxM = 1ull << 32;
constexpr uint32_t kMaxLeaves = 1u << 26;
constexpr uint32_t kMaxSlotsPerKey = 16;  // gapped RMI: slots per key of R

thread_local hipEvent_t t_ev_start = nullptr;
thread_local hipEvent_t t_ev_stop = nullptr;

// Workspace cache for the synchronous probe: one grow-only buffer per
// (device, stream).  Calls on one stream are ordered by the stream itself;
// growth frees the old buffer with hipFree, which waits for the device.
struct WsKey {
    int dev;
    hipStream_t stream;
    bool operator==(const WsKey& o) const { return dev == o.dev && stream == o.stream; }
};
struct WsKeyHash {
    size_t operator()(const WsKey& k) const {
        return std::hash<void*>()((void*)k.stream) ^ (size_t)k.dev * 0x9e3779b97f4a7c15ull;
    }
};
struct WsBuf {
    void* ptr = nullptr;
    uint64_t bytes = 0;
};
thread_local uint64_t* t_host_count = nullptr;  // pinned readback slot
std::mutex g_ws_mu;
std::unordered_map<WsKey, WsBuf, WsKeyHash> g_ws;

int check_device(const lj_index* idx) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LJ_ERR_DEVICE;
    return dev == idx->device ? LJ_OK : LJ_ERR_ARG;
}

int validate_build(const uint64_t* r, uint64_t n, uint32_t leaves, uint32_t flags) {
    if (n > 0 && !r) return LJ_ERR_ARG;
    if (leaves == 0) return LJ_ERR_ARG;
    if ((flags & ~31u) || ((flags & 3u) != LJ_LEAF_FP32 && (flags & 3u) != LJ_LEAF_FP64))
        return LJ_ERR_ARG;
    if (n >= kMaxN || leaves > kMaxLeaves) return LJ_ERR_TOO_LARGE;
    for (uint64_t i = 1; i < n; ++i)
        if (r[i - 1] > r[i]) return LJ_ERR_UNSORTED;
    return LJ_OK;
}

// What is built over the RMI: nothing (a plain RMI), gapped arrays or a
// learned hash table, with that many slots per key of R.
enum class Extra { kNone, kGapped, kHash };

int build_common(const uint64_t* r, uint64_t n, uint32_t leaves, uint32_t flags, Extra extra,
                 uint32_t slots_per_key, lj_index** out) {
    if (!out) return LJ_ERR_ARG;
    *out = nullptr;
    int st = validate_build(r, n, leaves, flags);
    if (st != LJ_OK) return st;
    lj_index* idx = new (std::nothrow) lj_index();
    if (!idx) return LJ_ERR_OOM;
    try {
        st = lj::fit_rmi(r, n, leaves, flags, idx);
        if (st == LJ_OK && extra == Extra::kGapped) st = lj::fit_gapped(r, slots_per_key, idx);
        if (st == LJ_OK && extra == Extra::kHash) st = lj::fit_hash(r, slots_per_key, idx);
    } catch (const std::bad_alloc&) {
        st = LJ_ERR_OOM;
    }
    if (st != LJ_OK) {
        delete idx;
        return st;
    }
    *out = idx;
    return LJ_OK;
}

int build_device(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves, uint32_t flags,
                 Extra extra, uint32_t slots_per_key, hipStream_t stream,
                 lj_index** out_index);

}  // namespace

extern "C" {

int lj_build_rmi_host_only(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                           uint32_t flags, lj_index** out_index) {
    int st = build_common(r_keys_host, n, leaves, flags, Extra::kNone, 0, out_index);
    if (st == LJ_OK) (*out_index)->host_only = true;
    return st;
}

int lj_build_gapped_rmi_host_only(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                                  uint32_t slots_per_key, uint32_t flags,
                                  lj_index** out_index) {
    if (out_index) *out_index = nullptr;
    if (slots_per_key < 1 || slots_per_key > kMaxSlotsPerKey) return LJ_ERR_ARG;
    int st = build_common(r_keys_host, n, leaves, flags, Extra::kGapped, slots_per_key,
                          out_index);
    if (st == LJ_OK) (*out_index)->host_only = true;
    return st;
}

int lj_build_learned_hash_host_only(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                                    uint32_t slots_per_key, uint32_t flags,
                                    lj_index** out_index) {
    if (out_index) *out_index = nullptr;
    if (slots_per_key < 1 || slots_per_key > kMaxSlotsPerKey) return LJ_ERR_ARG;
    int st = build_common(r_keys_host, n, leaves, flags, Extra::kHash, slots_per_key,
                          out_index);
    if (st == LJ_OK) (*out_index)->host_only = true;
    return st;
}

int lj_build_rmi(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves, uint32_t flags,
                 hipStream_t stream, lj_index** out_index) {
    return build_device(r_keys_host, n, leaves, flags, Extra::kNone, 0, stream, out_index);
}

int lj_build_gapped_rmi(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                        uint32_t slots_per_key, uint32_t flags, hipStream_t stream,
                        lj_index** out_index) {
    if (out_index) *out_index = nullptr;
    if (slots_per_key < 1 || slots_per_key > kMaxSlotsPerKey) return LJ_ERR_ARG;
    return build_device(r_keys_host, n, leaves, flags, Extra::kGapped, slots_per_key, stream,
                        out_index);
}

int lj_build_learned_hash(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                          uint32_t slots_per_key, uint32_t flags, hipStream_t stream,
                          lj_index** out_index) {
    if (out_index) *out_index = nullptr;
    if (slots_per_key < 1 || slots_per_key > kMaxSlotsPerKey) return LJ_ERR_ARG;
    return build_device(r_keys_host, n, leaves, flags, Extra::kHash, slots_per_key, stream,
                        out_index);
}

}  // extern "C"

namespace {

int build_device(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves, uint32_t flags,
                 Extra extra, uint32_t slots_per_key, hipStream_t stream,
                 lj_index** out_index) {
    int st = build_common(r_keys_host, n, leaves, flags, extra, slots_per_key, out_index);
    if (st != LJ_OK) return st;
    lj_index* idx = *out_index;
    *out_index = nullptr;
    if (hipGetDevice(&idx->device) != hipSuccess) {
        delete idx;
        return LJ_ERR_DEVICE;
    }
    const uint64_t rbytes = (n ? n : 1) * sizeof(uint64_t);
    const void* lsrc = lj::leaf_fp32(flags) ? (const void*)idx->leaf32.data()
                                             : (const void*)idx->leaf64.data();
    const uint64_t lbytes = (uint64_t)leaves * (lj::leaf_fp32(flags) ? sizeof(lj::LeafF32)
                                                                      : sizeof(lj::LeafF64));
    const uint64_t fbytes = idx->fences.size() * sizeof(uint64_t);
    const uint64_t bbytes = idx->bucket_lo.size() * sizeof(uint16_t);
    const uint64_t sbytes = idx->slots.size() * sizeof(lj::GSlot);
    const uint64_t hbytes = idx->buckets.size() * sizeof(lj::HBucket);
    const uint64_t nrs = (n + lj::kLineKeys - 1) / lj::kLineKeys;
    const uint64_t rsbytes = nrs * sizeof(uint64_t);
    const uint64_t tbytes = idx->root_tab.size() * sizeof(uint32_t);
    if (hipMalloc((void**)&idx->r_dev, rbytes) != hipSuccess ||
        hipMalloc(&idx->leaf_dev, lbytes) != hipSuccess ||
        (fbytes && hipMalloc((void**)&idx->fences_dev, fbytes) != hipSuccess) ||
        (bbytes && hipMalloc((void**)&idx->bucket_lo_dev, bbytes) != hipSuccess) ||
        (sbytes && hipMalloc((void**)&idx->slots_dev, sbytes) != hipSuccess) ||
        (hbytes && hipMalloc((void**)&idx->buckets_dev, hbytes) != hipSuccess) ||
        (rsbytes && hipMalloc((void**)&idx->rs_dev, rsbytes) != hipSuccess) ||
        (tbytes && hipMalloc((void**)&idx->root_tab_dev, tbytes) != hipSuccess)) {
        (void)hipGetLastError();
        lj_free_index(idx);
        return LJ_ERR_OOM;
    }
    idx->device_bytes = rbytes + lbytes + fbytes + bbytes + sbytes + hbytes + rsbytes + tbytes;
    idx->root.tab_dev = idx->root_tab_dev;
    hipError_t e = hipSuccess;
    if (n) e = hipMemcpyAsync(idx->r_dev, r_keys_host, n * sizeof(uint64_t),
                              hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(idx->leaf_dev, lsrc, lbytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && fbytes)
        e = hipMemcpyAsync(idx->fences_dev, idx->fences.data(), fbytes, hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess && bbytes)
        e = hipMemcpyAsync(idx->bucket_lo_dev, idx->bucket_lo.data(), bbytes,
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && sbytes)
        e = hipMemcpyAsync(idx->slots_dev, idx->slots.data(), sbytes, hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess && hbytes)
        e = hipMemcpyAsync(idx->buckets_dev, idx->buckets.data(), hbytes, hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess && tbytes)
        e = hipMemcpyAsync(idx->root_tab_dev, idx->root_tab.data(), tbytes,
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && rsbytes)
        e = lj::launch_line_samples(idx->r_dev, n, idx->rs_dev, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        lj_free_index(idx);
        return LJ_ERR_DEVICE;
    }
    std::vector<lj::GSlot>().swap(idx->slots);  // the device copies are the ones probed
    std::vector<lj::HBucket>().swap(idx->buckets);
    *out_index = idx;
    return LJ_OK;
}

}  // namespace

extern "C" {

void lj_free_index(lj_index* idx) {
    if (!idx) return;
    if (idx->r_dev) (void)hipFree(idx->r_dev);
    if (idx->leaf_dev) (void)hipFree(idx->leaf_dev);
    if (idx->fences_dev) (void)hipFree(idx->fences_dev);
    if (idx->bucket_lo_dev) (void)hipFree(idx->bucket_lo_dev);
    if (idx->slots_dev) (void)hipFree(idx->slots_dev);
    if (idx->buckets_dev) (void)hipFree(idx->buckets_dev);
    if (idx->rs_dev) (void)hipFree(idx->rs_dev);
    if (idx->root_tab_dev) (void)hipFree(idx->root_tab_dev);
    delete idx;
}

uint64_t lj_probe_workspace_bytes(const lj_index* idx, uint64_t m) {
    return idx ? lj::ws_bytes(idx, m) : 0;
}

int lj_probe_set_timing_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
    return LJ_OK;
}

int lj_probe_join_async(const lj_index* idx, const uint64_t* s, uint64_t m, lj_pair* out,
                        uint64_t cap, uint64_t* count_dev, void* ws, uint64_t ws_bytes,
                        hipStream_t stream) {
    hipEvent_t ev0 = t_ev_start, ev1 = t_ev_stop;
    t_ev_start = t_ev_stop = nullptr;
    if (!idx || idx->host_only || !count_dev) return LJ_ERR_ARG;
    if (m > 0 && !s) return LJ_ERR_ARG;
    if (cap > 0 && !out) return LJ_ERR_ARG;
    if (m >= kMaxM) return LJ_ERR_TOO_LARGE;
    int st = check_device(idx);
    if (st != LJ_OK) return st;
    if (m == 0) return lj::launch_set_u64(count_dev, 0, stream) == hipSuccess ? LJ_OK
                                                                             : LJ_ERR_DEVICE;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < lj::ws_bytes(idx, m))
        return LJ_ERR_WORKSPACE;
    hipError_t e = lj::launch_probe(idx, s, m, out, cap, count_dev, ws, stream, ev0, ev1);
    return e == hipSuccess ? LJ_OK : LJ_ERR_DEVICE;
}

int lj_probe_join(const lj_index* idx, const uint64_t* s, uint64_t m, lj_pair* out,
                  uint64_t cap, uint64_t* count_host, hipStream_t stream) {
    hipEvent_t ev0 = t_ev_start, ev1 = t_ev_stop;
    t_ev_start = t_ev_stop = nullptr;
    if (!idx || idx->host_only || !count_host) return LJ_ERR_ARG;
    if (m > 0 && !s) return LJ_ERR_ARG;
    if (cap > 0 && !out) return LJ_ERR_ARG;
    if (m >= kMaxM) return LJ_ERR_TOO_LARGE;
    int st = check_device(idx);
    if (st != LJ_OK) return st;
    if (m == 0) {
        *count_host = 0;
        return LJ_OK;
    }
    const uint64_t need = lj::ws_bytes(idx, m);
    if (!t_host_count) {
        if (hipHostMalloc((void**)&t_host_count, sizeof(uint64_t)) != hipSuccess) {
            t_host_count = nullptr;
            return LJ_ERR_OOM;
        }
    }
    hipError_t e;
    {
        // Hold the lock until the work is enqueued, so that a concurrent
        // growth (whose hipFree waits for the device) cannot free a buffer
        // this call is about to use.
        std::lock_guard<std::mutex> lock(g_ws_mu);
        WsBuf& wb = g_ws[WsKey{idx->device, stream}];
        if (wb.bytes < need) {
            if (wb.ptr) (void)hipFree(wb.ptr);
            wb.ptr = nullptr;
            wb.bytes = 0;
            uint64_t sz = need + need / 4;
            if (hipMalloc(&wb.ptr, sz) != hipSuccess) {
                (void)hipGetLastError();
                wb.ptr = nullptr;
                return LJ_ERR_OOM;
            }
            wb.bytes = sz;
        }
        uint64_t* cnt_dev = &((lj::WsHeader*)wb.ptr)->count;
        e = lj::launch_probe(idx, s, m, out, cap, cnt_dev, wb.ptr, stream, ev0, ev1);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t_host_count, cnt_dev, sizeof(uint64_t), hipMemcpyDeviceToHost,
                               stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return LJ_ERR_DEVICE;
    const uint64_t total = *t_host_count;
    if (total == ~0ull) return LJ_ERR_DEVICE;
    *count_host = total;
    // A count-only probe (no output buffer) is not a capacity error.
    return (out && total > cap) ? LJ_ERR_CAPACITY : LJ_OK;
}

uint64_t lj_sort_join_workspace_bytes(uint64_t n, uint64_t m) {
    return lj::sort_join_ws(n, m).total;
}

int lj_learned_sort_async(const uint64_t* keys, uint64_t n, uint64_t* keys_out,
                          uint32_t* pos_out, void* ws, uint64_t ws_bytes, hipStream_t stream) {
    if (n > 0 && (!keys || !keys_out || !pos_out)) return LJ_ERR_ARG;
    if (n >= kMaxN) return LJ_ERR_TOO_LARGE;
    if (n == 0) return LJ_OK;
    const lj::SortJoinWs L = lj::sort_join_ws(n, 0);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < L.total) return LJ_ERR_WORKSPACE;
    return lj::launch_learned_sort(keys, n, keys_out, pos_out, ws, L, stream) == hipSuccess
               ? LJ_OK
               : LJ_ERR_DEVICE;
}

int lj_sort_join_async(const uint64_t* r, uint64_t n, const uint64_t* s, uint64_t m,
                       lj_pair* out, uint64_t cap, uint64_t* count_dev, void* ws,
                       uint64_t ws_bytes, hipStream_t stream) {
    hipEvent_t ev0 = t_ev_start, ev1 = t_ev_stop;
    t_ev_start = t_ev_stop = nullptr;
    if (!count_dev || (n > 0 && !r) || (m > 0 && !s) || (cap > 0 && !out)) return LJ_ERR_ARG;
    if (n >= kMaxN || m >= kMaxM) return LJ_ERR_TOO_LARGE;
    if (n > 0 && m > 0 &&
        (!ws || ((uintptr_t)ws & 255) || ws_bytes < lj::sort_join_ws(n, m).total))
        return LJ_ERR_WORKSPACE;
    return lj::launch_sort_join(r, n, s, m, out, cap, count_dev, ws, stream, ev0, ev1) ==
                   hipSuccess
               ? LJ_OK
               : LJ_ERR_DEVICE;
}

int lj_index_get_stats(const lj_index* idx, lj_index_stats* o) {
    if (!idx || !o) return LJ_ERR_ARG;
    o->n = idx->n;
    o->leaves = idx->leaves;
    o->flags = idx->flags;
    o->nonempty_leaves = idx->nonempty_leaves;
    o->max_leaf_keys = idx->max_leaf_keys;
    o->max_mult = idx->max_mult;
    o->mean_window = idx->mean_window;
    o->max_window = idx->max_window;
    o->device_bytes = idx->device_bytes;
    o->root_a0 = idx->root.a0;
    o->root_b0 = idx->root.b0;
    o->root_kmin = idx->root.kmin;
    o->slots_per_key = idx->gap ? idx->gap : idx->hash_spk;
    o->pad = 0;
    o->nslots = idx->gap ? idx->nslots : idx->nbuckets * lj::kBucketSlots;
    return LJ_OK;
}

int lj_gapped_slots_host(const lj_index* idx, uint64_t* keys, uint32_t* ridx, uint64_t cap,
                         uint64_t* nslots_out) {
    if (!idx || !idx->gap || idx->slots.size() != idx->nslots || !nslots_out) return LJ_ERR_ARG;
    if (cap && (!keys || !ridx)) return LJ_ERR_ARG;
    *nslots_out = idx->nslots;
    const uint64_t k = std::min<uint64_t>(cap, idx->nslots);
    for (uint64_t j = 0; j < k; ++j) {
        keys[j] = idx->slots[j].key;
        ridx[j] = idx->slots[j].ridx;
    }
    return cap >= idx->nslots ? LJ_OK : LJ_ERR_CAPACITY;
}

int lj_hash_buckets_host(const lj_index* idx, uint64_t* keys, uint32_t* ridx, uint32_t* next,
                         uint64_t cap, uint64_t* nbuckets_out, uint64_t* nprimary_out) {
    if (!idx || !idx->hash_spk || idx->buckets.size() != idx->nbuckets || !nbuckets_out)
        return LJ_ERR_ARG;
    if (cap && (!keys || !ridx || !next)) return LJ_ERR_ARG;
    *nbuckets_out = idx->nbuckets;
    if (nprimary_out) *nprimary_out = idx->nprimary;
    const uint64_t k = std::min<uint64_t>(cap, idx->nbuckets);
    for (uint64_t b = 0; b < k; ++b) {
        const lj::HBucket& h = idx->buckets[b];
        for (uint32_t j = 0; j < lj::kBucketSlots; ++j) {
            keys[b * lj::kBucketSlots + j] = j < h.nkeys ? h.key[j] : 0;
            ridx[b * lj::kBucketSlots + j] = j < h.nkeys ? h.ridx[j] : lj::kGap;
        }
        next[b] = h.next;
    }
    return cap >= idx->nbuckets ? LJ_OK : LJ_ERR_CAPACITY;
}

int lj_self_check(const lj_index* idx, uint64_t* viol_host, hipStream_t stream) {
    if (!idx || idx->host_only || !viol_host) return LJ_ERR_ARG;
    int st = check_device(idx);
    if (st != LJ_OK) return st;
    uint64_t* d = nullptr;  // violations, and a gapped index's key-slot count
    if (hipMalloc((void**)&d, 2 * sizeof(uint64_t)) != hipSuccess) return LJ_ERR_OOM;
    hipError_t e = lj::launch_self_check(idx, d, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(viol_host, d, sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(d);
    return e == hipSuccess ? LJ_OK : LJ_ERR_DEVICE;
}

int lj_predict_windows(const lj_index* idx, const uint64_t* keys, uint64_t m, uint32_t* leaf,
                       int64_t* pred, int64_t* wlo, int64_t* whi, hipStream_t stream) {
    if (!idx || idx->host_only || (m && !keys)) return LJ_ERR_ARG;
    int st = check_device(idx);
    if (st != LJ_OK) return st;
    return lj::launch_predict_windows(idx, keys, m, leaf, pred, wlo, whi, stream) == hipSuccess
               ? LJ_OK
               : LJ_ERR_DEVICE;
}

int lj_predict_windows_host(const lj_index* idx, const uint64_t* keys, uint64_t m,
                            uint32_t* leaf, int64_t* pred, int64_t* wlo, int64_t* whi) {
    if (!idx || (m && !keys)) return LJ_ERR_ARG;
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t x = keys[i];
        uint32_t l = lj::route(idx->root, x);
        int64_t lo = 1, hi = 0, pr = -1;
        uint32_t cnt = 0, pos0 = 0;
        int32_t elo = 0, ehi = 0, rel = 0;
        if (lj::leaf_fp32(idx->flags)) {
            const lj::LeafF32& lf = idx->leaf32[l];
            cnt = lf.cnt;
            if (cnt) rel = lj::predict_rel(lf, x);
            pos0 = lf.pos0;
            elo = lf.lo;
            ehi = lf.hi;
        } else {
            const lj::LeafF64& lf = idx->leaf64[l];
            cnt = lf.cnt;
            if (cnt) rel = lj::predict_rel(lf, x);
            pos0 = lf.pos0;
            elo = lf.lo;
            ehi = lf.hi;
        }
        if (cnt && idx->hash_spk) {
            // Learned hash: the primary bucket.
            int64_t rc = rel < 0 ? 0 : (rel > (int64_t)cnt - 1 ? (int64_t)cnt - 1 : rel);
            pr = (((int64_t)pos0 + rc) * (int64_t)idx->hash_spk) / (int64_t)lj::kBucketSlots;
            lo = hi = pr;
        } else if (cnt && idx->gap) {
            // Gapped index: slot window [s, s + hi] of the predicted slot s.
            int64_t rc = rel < 0 ? 0 : (rel > (int64_t)cnt - 1 ? (int64_t)cnt - 1 : rel);
            pr = ((int64_t)pos0 + rc) * (int64_t)idx->gap;
            lo = pr;
            hi = std::min<int64_t>(pr + ehi, (int64_t)idx->nslots - 1);
        } else if (cnt) {
            pr = (int64_t)pos0 + rel;
            int64_t a = (int64_t)rel + elo, b = (int64_t)rel + ehi;
            if (a < 0) a = 0;
            if (b > (int64_t)cnt - 1) b = (int64_t)cnt - 1;
            if (a <= b) {
                lo = (int64_t)pos0 + a;
                hi = (int64_t)pos0 + b;
            }
        }
        if (leaf) leaf[i] = l;
        if (pred) pred[i] = pr;
        if (wlo) wlo[i] = lo;
        if (whi) whi[i] = hi;
    }
    return LJ_OK;
}

int lj_bench_random_gather(const void* buf, uint64_t bytes, uint32_t granule, uint64_t reads,
                           uint64_t seed, uint64_t* sink, hipStream_t stream) {
    if (!buf || !sink || granule < 8 || granule > 4096 || (granule & (granule - 1)) ||
        bytes < granule)
        return LJ_ERR_ARG;
    return lj::launch_random_gather(buf, bytes, granule, reads, seed, sink, stream) ==
                   hipSuccess
               ? LJ_OK
               : LJ_ERR_DEVICE;
}

const char* lj_strerror(int s) {
    switch (s) {
        case LJ_OK: return "ok";
        case LJ_ERR_ARG: return "invalid argument";
        case LJ_ERR_UNSORTED: return "inner relation is not sorted";
        case LJ_ERR_TOO_LARGE: return "size beyond the supported range";
        case LJ_ERR_CAPACITY: return "output capacity too small";
        case LJ_ERR_DEVICE: return "device error";
        case LJ_ERR_OOM: return "out of memory";
        case LJ_ERR_WORKSPACE: return "workspace too small or misaligned";
        case LJ_ERR_TIMEOUT: return "timed out";
        default: return "unknown status";
    }
}

}  // extern "C"
