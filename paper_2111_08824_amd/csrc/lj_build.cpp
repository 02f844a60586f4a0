// Host-side construction of the two-level linear RMI (Section II-D,
// "Recursive Model Index"): FP64 least-squares fits of the root and of every
// leaf, then per-leaf min/max error bounds recomputed under the exact probe
// arithmetic of rmi_eval.h.  Building is offline and untimed (Section III-A,
// "GRMI Building": the index exists before the join).
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "lj_internal.h"

namespace lj {
namespace {

// Run body(begin, end) over [0, total) split into contiguous chunks, one per
// hardware thread.
template <class F>
void parallel_chunks(uint64_t total, F body) {
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (total < (1u << 16) || nt == 1) {
        body(0, total);
        return;
    }
    std::vector<std::thread> th;
    uint64_t step = (total + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        uint64_t b = t * step, e = std::min(total, b + step);
        if (b >= e) break;
        th.emplace_back([=] { body(b, e); });
    }
    for (auto& x : th) x.join();
}

// Run body(i) for i in [0, count) with dynamic scheduling.
template <class F>
void parallel_items(uint64_t count, F body) {
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (count < 64 || nt == 1) {
        for (uint64_t i = 0; i < count; ++i) body(i);
        return;
    }
    std::atomic<uint64_t> next{0};
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (;;) {
                uint64_t b = next.fetch_add(256);
                if (b >= count) break;
                uint64_t e = std::min(count, b + 256);
                for (uint64_t i = b; i < e; ++i) body(i);
            }
        });
    for (auto& x : th) x.join();
}

struct Fit {
    double slope, icpt;
};

// Least squares y = icpt + slope * x over points (x_i, y_i), centred two-pass
// sums.  A degenerate set (all x equal) gets slope 0 and the mean of y.
template <class X, class Y>
Fit ols(uint64_t cnt, X x, Y y) {
    double mx = 0, my = 0;
    for (uint64_t i = 0; i < cnt; ++i) {
        mx += x(i);
        my += y(i);
    }
    mx /= (double)cnt;
    my /= (double)cnt;
    double sxx = 0, sxy = 0;
    for (uint64_t i = 0; i < cnt; ++i) {
        double dx = x(i) - mx;
        sxx += dx * dx;
        sxy += dx * (y(i) - my);
    }
    double b = (sxx > 0 && sxy > 0) ? sxy / sxx : 0.0;
    return {b, my - b * mx};
}

template <class Leaf>
void fit_leaves(const uint64_t* r, const std::vector<uint64_t>& pos0,
                const std::vector<uint64_t>& cnt, uint32_t L, std::vector<Leaf>& out) {
    out.assign(L, Leaf{});
    parallel_items(L, [&](uint64_t l) {
        Leaf lf{};
        lf.pos0 = (uint32_t)pos0[l];
        lf.cnt = (uint32_t)cnt[l];
        if (cnt[l] == 0) {
            lf.lo = 1;  // empty window marker (lo > hi); never searched
            lf.hi = 0;
            out[l] = lf;
            return;
        }
        const uint64_t* k = r + pos0[l];
        lf.base = k[0];
        Fit f = ols(cnt[l], [&](uint64_t i) { return u64_to_f64(k[i] - k[0]); },
                    [&](uint64_t i) { return (double)i; });
        lf.slope = (decltype(lf.slope))f.slope;
        lf.icpt = (decltype(lf.icpt))f.icpt;
        // Error bounds under the probe's own arithmetic.
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (uint64_t i = 0; i < cnt[l]; ++i) {
            int64_t e = (int64_t)i - (int64_t)predict_rel(lf, k[i]);
            lo = std::min(lo, e);
            hi = std::max(hi, e);
        }
        lf.lo = (int32_t)lo;
        lf.hi = (int32_t)hi;
        out[l] = lf;
    });
}

// Search-window statistics over the keys of R (an RMI's windows are clipped
// to the leaf's run; a gapped index's slot windows are not).
template <class Leaf>
void leaf_stats(const std::vector<Leaf>& lv, lj_index* idx, bool clip_to_run = true) {
    double wsum = 0;
    uint64_t wmax = 0;
    uint32_t ne = 0, mk = 0;
    for (const Leaf& lf : lv) {
        if (lf.cnt == 0) continue;
        ++ne;
        mk = std::max(mk, lf.cnt);
        uint64_t w = (uint64_t)((int64_t)lf.hi - (int64_t)lf.lo + 1);
        if (clip_to_run) w = std::min<uint64_t>(w, lf.cnt);
        wsum += (double)w * lf.cnt;
        wmax = std::max(wmax, w);
    }
    idx->nonempty_leaves = ne;
    idx->max_leaf_keys = mk;
    idx->mean_window = idx->n ? wsum / (double)idx->n : 0.0;
    idx->max_window = wmax;
}

}  // namespace

int fit_rmi(const uint64_t* r, uint64_t n, uint32_t L, uint32_t flags, lj_index* idx) {
    idx->n = n;
    idx->leaves = L;
    idx->flags = flags;

    RootModel rm{};
    rm.leaves = L;
    if (flags & LJ_ROOT_RADIX) {
        // Radix root: the leaf coordinate L * rank / n of every bucket's
        // lower edge, rank = keys of R below it (fixed point with as many
        // fraction bits as keep L << frac_bits below 2^31).
        rm.kind = kRootRadix;
        rm.kmin = n ? r[0] : 0;
        uint32_t lg = 0;
        while ((1ull << lg) < L) ++lg;
        rm.frac_bits = 31 - lg;
        const uint64_t full = (uint64_t)L << rm.frac_bits;
        std::vector<uint32_t>& tab = idx->root_tab;
        tab.assign(kRootTabLen, (uint32_t)full);
        for (uint32_t b = 0; b < kRootBuckets && n > 0; ++b) {
            // Lower edge of bucket b as an offset from kmin.
            unsigned __int128 edge;
            if (b < (1u << kRootSubBits)) {
                edge = b;
            } else {
                const uint32_t e = (b >> kRootSubBits) + kRootSubBits - 1;
                const uint32_t sub = b & ((1u << kRootSubBits) - 1);
                edge = (unsigned __int128)((1u << kRootSubBits) + sub) << (e - kRootSubBits);
            }
            const unsigned __int128 key = (unsigned __int128)rm.kmin + edge;
            uint64_t rank = n;
            if (key <= (unsigned __int128)~0ull)
                rank = (uint64_t)(std::lower_bound(r, r + n, (uint64_t)key) - r);
            tab[b] = (uint32_t)(((unsigned __int128)rank * full) / n);
        }
        rm.tab_host = tab.data();
    } else if (n > 0) {
        // Linear root: least squares from (key - R[0]) to the leaf
        // coordinate i*L/n.
        rm.kmin = r[0];
        const double scale = (double)L / (double)n;
        Fit f = ols(n, [&](uint64_t i) { return u64_to_f64(r[i] - r[0]); },
                    [&](uint64_t i) { return (double)i * scale; });
        rm.a0 = f.icpt;
        rm.b0 = f.slope;  // >= 0: keys are sorted, so the covariance is >= 0
    }
    idx->root = rm;

    // Route every key; routing is non-decreasing in the key, so each leaf
    // owns one contiguous run of R.
    std::vector<uint32_t> leaf_of(n);
    parallel_chunks(n, [&](uint64_t b, uint64_t e) {
        for (uint64_t i = b; i < e; ++i) leaf_of[i] = route(rm, r[i]);
    });
    std::vector<uint64_t> pos0(L, 0), cnt(L, 0);
    for (uint64_t i = 0; i < n; ++i) {
        if (i > 0 && leaf_of[i] < leaf_of[i - 1]) return LJ_ERR_DEVICE;  // cannot happen
        cnt[leaf_of[i]]++;
    }
    uint64_t acc = 0;
    for (uint32_t l = 0; l < L; ++l) {
        pos0[l] = acc;
        acc += cnt[l];
    }
    leaf_of.clear();
    leaf_of.shrink_to_fit();

    // Longest run of equal keys.
    uint64_t mm = n ? 1 : 0, run = 1;
    for (uint64_t i = 1; i < n; ++i) {
        run = (r[i] == r[i - 1]) ? run + 1 : 1;
        mm = std::max(mm, run);
    }
    idx->max_mult = mm;

    // Equi-depth key ranges of R for the binned probe (built for every
    // index, 61 KB, so that batched plans can choose the binned probe).
    if (n > 0) {
        idx->fences.resize(kBins - 1);
        for (uint32_t i = 0; i + 1 < kBins; ++i)
            idx->fences[i] = r[((uint64_t)(i + 1) * n) / kBins];
        idx->bucket_lo.assign(kBuckets + 1, 0);
        for (uint64_t f : idx->fences) idx->bucket_lo[key_bucket(f) + 1]++;
        for (uint32_t b = 0; b < kBuckets; ++b) idx->bucket_lo[b + 1] += idx->bucket_lo[b];
    }

    if (leaf_fp32(flags)) {
        fit_leaves(r, pos0, cnt, L, idx->leaf32);
        leaf_stats(idx->leaf32, idx);
    } else {
        fit_leaves(r, pos0, cnt, L, idx->leaf64);
        leaf_stats(idx->leaf64, idx);
    }
    return LJ_OK;
}

namespace {

// Model-based insertion for one leaf arithmetic (Section III-A, "GRMI
// Building": the RMI built over R places every key in the gapped array).
template <class Leaf>
int fit_gapped_leaves(const uint64_t* r, uint32_t G, std::vector<Leaf>& lv, lj_index* idx) {
    const uint64_t n = idx->n;
    // Predicted slot of every key; keys go in order, each to its predicted
    // slot or, when taken, to the slot after the previous key, so the array
    // stays sorted and equal keys stay adjacent.
    std::vector<uint64_t> slot(n);
    parallel_items(lv.size(), [&](uint64_t l) {
        const Leaf& lf = lv[l];
        for (uint64_t i = lf.pos0; i < (uint64_t)lf.pos0 + lf.cnt; ++i)
            slot[i] = gapped_pred(lf, r[i], G);
    });
    uint64_t prev = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t pred = slot[i];
        slot[i] = (i == 0 || pred > prev) ? pred : prev + 1;
        prev = slot[i];
    }
    const uint64_t nslots = n ? std::max<uint64_t>(n * G, slot[n - 1] + 1) : 1;
    if (nslots >= (1ull << 32)) return LJ_ERR_TOO_LARGE;
    // Per leaf: the largest distance from a key's predicted slot to its slot.
    parallel_items(lv.size(), [&](uint64_t l) {
        Leaf& lf = lv[l];
        if (lf.cnt == 0) return;  // keeps lo > hi: empty
        uint64_t drift = 0;
        for (uint64_t i = lf.pos0; i < (uint64_t)lf.pos0 + lf.cnt; ++i)
            drift = std::max(drift, slot[i] - gapped_pred(lf, r[i], G));
        lf.lo = 0;
        lf.hi = (int32_t)std::min<uint64_t>(drift, 0x7FFFFFFF);
    });
    // Fill: keys with their positions; gaps with the next key of R.
    idx->slots.assign(nslots, GSlot{~0ull, kGap, 0u});
    for (uint64_t i = 0; i < n; ++i) idx->slots[slot[i]] = GSlot{r[i], (uint32_t)i, 0u};
    uint64_t next = ~0ull;
    for (uint64_t j = nslots; j-- > 0;) {
        if (idx->slots[j].ridx != kGap) next = idx->slots[j].key;
        else idx->slots[j].key = next;
    }
    idx->nslots = nslots;
    idx->gap = G;
    leaf_stats(lv, idx, false);
    return LJ_OK;
}

// Learned hash table for one leaf arithmetic (Section III-C): the RMI's
// position estimate is the hash; keys of R go, in order, to the end of
// their bucket's chain, so each chain lists its keys in R order and all
// copies of a key share one chain.
template <class Leaf>
int fit_hash_leaves(const uint64_t* r, uint32_t spk, const std::vector<Leaf>& lv,
                    lj_index* idx) {
    const uint64_t n = idx->n;
    const uint64_t nprimary = n ? ((n - 1) * spk) / kBucketSlots + 1 : 1;
    if (nprimary >= kNoBucket) return LJ_ERR_TOO_LARGE;
    std::vector<uint64_t> bucket(n);
    parallel_items(lv.size(), [&](uint64_t l) {
        const Leaf& lf = lv[l];
        for (uint64_t i = lf.pos0; i < (uint64_t)lf.pos0 + lf.cnt; ++i)
            bucket[i] = hash_bucket(lf, r[i], spk);
    });
    std::vector<HBucket>& B = idx->buckets;
    B.assign(nprimary, HBucket{{0, 0, 0, 0}, {kGap, kGap, kGap, kGap}, kNoBucket, 0u, {0u, 0u}});
    std::vector<uint32_t> tail(nprimary);
    for (uint64_t b = 0; b < nprimary; ++b) tail[b] = (uint32_t)b;
    double depth_sum = 0;
    uint64_t depth_max = 0;
    std::vector<uint32_t> depth(nprimary, 1);  // chain length of each primary bucket
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t b = bucket[i];
        uint32_t t = tail[b];
        if (B[t].nkeys == kBucketSlots) {
            if (B.size() >= kNoBucket) return LJ_ERR_TOO_LARGE;
            const uint32_t nb = (uint32_t)B.size();
            B.push_back(HBucket{{0, 0, 0, 0}, {kGap, kGap, kGap, kGap}, kNoBucket, 0u, {0u, 0u}});
            B[t].next = nb;
            tail[b] = t = nb;
            ++depth[b];
        }
        HBucket& h = B[t];
        h.key[h.nkeys] = r[i];
        h.ridx[h.nkeys] = (uint32_t)i;
        ++h.nkeys;
        depth_sum += depth[b];
        depth_max = std::max<uint64_t>(depth_max, depth[b]);
    }
    idx->nprimary = nprimary;
    idx->nbuckets = B.size();
    idx->hash_spk = spk;
    // Window statistics in buckets: chain position of each key of R.
    idx->mean_window = n ? depth_sum / (double)n : 0.0;
    idx->max_window = depth_max;
    return LJ_OK;
}

}  // namespace

int fit_hash(const uint64_t* r, uint32_t spk, lj_index* idx) {
    if (spk < 1) return LJ_ERR_ARG;
    return leaf_fp32(idx->flags) ? fit_hash_leaves(r, spk, idx->leaf32, idx)
                                 : fit_hash_leaves(r, spk, idx->leaf64, idx);
}

int fit_gapped(const uint64_t* r, uint32_t G, lj_index* idx) {
    if (G < 1) return LJ_ERR_ARG;
    return leaf_fp32(idx->flags) ? fit_gapped_leaves(r, G, idx->leaf32, idx)
                                 : fit_gapped_leaves(r, G, idx->leaf64, idx);
}

}  // namespace lj
