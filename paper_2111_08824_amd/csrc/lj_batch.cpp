// Batched probe: plan objects that enqueue one fused probe kernel per batch,
// spread over parallel branches (fork/join across streams), optionally
// captured once into a HIP graph and replayed; and the autotuner that picks
// their launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "lj_batch.h"

// Batches probed directly on plain RMIs with one leaf arithmetic and
// duplicate class, run by one fused launch: their jobs (device table in the
// plan's workspace), tiles and branch.
struct FusedGroup {
    int group = 0;
    uint64_t jobs_off = 0;  // FusedJob table
    uint64_t hdr_off = 0;   // launch header
    uint32_t njobs = 0;
    uint32_t tiles = 0;
    uint64_t keys = 0;
    uint32_t branch = 0;
};

struct lj_batch_plan {
    int device = -1;
    std::vector<lj_batch_desc> descs;
    std::vector<uint64_t> ws_off;    // per batch workspace offset
    std::vector<uint32_t> kpl;       // per batch keys per lane
    std::vector<int> mode;           // per batch probe form (see uses_binned)
    std::vector<int> fused;          // per batch fused group slot, or -1
    std::vector<uint32_t> branch;    // per batch branch
    std::vector<FusedGroup> groups;
    void* ws = nullptr;
    uint32_t branches = 1;
    std::vector<hipStream_t> streams;  // one per branch
    std::vector<hipEvent_t> join;      // one per branch
    hipEvent_t fork = nullptr;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace lj {

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

namespace {

bool kpl_allowed(uint32_t k) { return k == 4 || k == 8 || k == 16 || k == 24; }

}  // namespace

int size_class(uint64_t m) {
    if (m < (1ull << 13)) return 0;
    if (m < (1ull << 17)) return 1;
    if (m < (1ull << 21)) return 2;
    return 3;
}

void default_tuning(lj_batch_tuning* t) {
    t->keys_per_lane[0] = 4;
    t->keys_per_lane[1] = 8;
    t->keys_per_lane[2] = 8;
    t->keys_per_lane[3] = 8;
    t->branches = 4;
    t->use_graph = 1;
    t->binned_min_keys = 0;
    t->measured_ms = 0.f;
    t->fused = 1;
}

int validate_tuning(const lj_batch_tuning& t) {
    for (int c = 0; c < 4; ++c)
        if (!kpl_allowed(t.keys_per_lane[c])) return LJ_ERR_ARG;
    if (t.branches < 1 || t.branches > kMaxBranches) return LJ_ERR_ARG;
    if (t.fused > 1) return LJ_ERR_ARG;
    return LJ_OK;
}

int validate_descs(const lj_batch_desc* d, uint32_t k, int device) {
    if (!d || k == 0) return LJ_ERR_ARG;
    for (uint32_t b = 0; b < k; ++b) {
        const lj_index* idx = d[b].index;
        if (!idx || idx->host_only || idx->device != device || !d[b].out_count_dev)
            return LJ_ERR_ARG;
        if (d[b].m > 0 && !d[b].s_keys_dev) return LJ_ERR_ARG;
        if (d[b].out_capacity > 0 && !d[b].out_pairs_dev) return LJ_ERR_ARG;
        if (d[b].m >= (1ull << 32)) return LJ_ERR_TOO_LARGE;
    }
    return LJ_OK;
}

int batch_mode(const lj_batch_tuning& t, uint64_t m) {
    if (t.binned_min_keys == 0) return -1;
    return m >= t.binned_min_keys ? 1 : 0;
}

hipError_t enqueue_one(const lj_batch_desc& d, void* ws, uint32_t kpl, int mode,
                       hipStream_t st) {
    if (d.m == 0) return launch_set_u64(d.out_count_dev, 0, st);
    if (d.index->max_mult > 1) kpl = std::min<uint32_t>(kpl, kItemsDupMax);
    return launch_probe(d.index, d.s_keys_dev, d.m, d.out_pairs_dev,
                        d.out_pairs_dev ? d.out_capacity : 0, d.out_count_dev, ws, st, nullptr,
                        nullptr, kpl, mode);
}

}  // namespace lj

namespace {

// Enqueue every batch of the plan, forked from `stream` over the branch
// streams and joined back into it.
hipError_t enqueue_fused(lj_batch_plan* p, const FusedGroup& g, hipStream_t st) {
    char* w = (char*)p->ws;
    return lj::launch_probe_fused((const lj::FusedJob*)(w + g.jobs_off), g.njobs, g.tiles,
                                  g.group, (uint32_t*)(w + g.hdr_off), st);
}

hipError_t enqueue_plan(lj_batch_plan* p, hipStream_t stream) {
    const size_t k = p->descs.size();
    if (p->branches == 1) {
        hipError_t e = hipSuccess;
        for (const FusedGroup& g : p->groups)
            if (e == hipSuccess) e = enqueue_fused(p, g, stream);
        for (size_t b = 0; b < k && e == hipSuccess; ++b) {
            if (p->fused[b] >= 0) continue;
            e = lj::enqueue_one(p->descs[b], (char*)p->ws + p->ws_off[b], p->kpl[b],
                                p->mode[b], stream);
        }
        return e;
    }
    hipError_t e = hipEventRecord(p->fork, stream);
    for (uint32_t r = 0; r < p->branches && e == hipSuccess; ++r)
        e = hipStreamWaitEvent(p->streams[r], p->fork, 0);
    for (const FusedGroup& g : p->groups)
        if (e == hipSuccess) e = enqueue_fused(p, g, p->streams[g.branch]);
    for (size_t b = 0; b < k && e == hipSuccess; ++b) {
        if (p->fused[b] >= 0) continue;
        e = lj::enqueue_one(p->descs[b], (char*)p->ws + p->ws_off[b], p->kpl[b], p->mode[b],
                            p->streams[p->branch[b]]);
    }
    for (uint32_t r = 0; r < p->branches && e == hipSuccess; ++r) {
        e = hipEventRecord(p->join[r], p->streams[r]);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, p->join[r], 0);
    }
    return e;
}

int plan_create(const lj_batch_desc* descs, uint32_t k, const lj_batch_tuning* tuning,
                lj_batch_plan** out) {
    if (!out) return LJ_ERR_ARG;
    *out = nullptr;
    lj_batch_tuning t;
    if (tuning) t = *tuning;
    else lj::default_tuning(&t);
    int st = lj::validate_tuning(t);
    if (st != LJ_OK) return st;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LJ_ERR_DEVICE;
    st = lj::validate_descs(descs, k, dev);
    if (st != LJ_OK) return st;

    lj_batch_plan* p = new (std::nothrow) lj_batch_plan();
    if (!p) return LJ_ERR_OOM;
    p->device = dev;
    p->descs.assign(descs, descs + k);
    p->branches = std::min<uint32_t>(t.branches, k);
    p->use_graph = t.use_graph != 0;

    // Workspace slices, keys per lane and probe form; batches that take the
    // direct probe on a plain RMI join their group's fused launch (when
    // t.fused), larger batches first in the group's tile-id space.
    std::vector<uint32_t> order(k);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return descs[a].m > descs[b].m; });
    uint64_t off = 0;
    p->ws_off.assign(k, 0);
    p->kpl.assign(k, 0);
    p->mode.assign(k, 0);
    p->fused.assign(k, -1);
    int slot_of_group[lj::kFusedGroups];
    std::fill(slot_of_group, slot_of_group + lj::kFusedGroups, -1);
    for (uint32_t b : order) {
        const lj_index* idx = descs[b].index;
        p->kpl[b] = t.keys_per_lane[lj::size_class(descs[b].m)];
        p->mode[b] = lj::batch_mode(t, descs[b].m);
        const int g = lj::fused_group(idx);
        if (t.fused && descs[b].m > 0 && g >= 0 && !lj::uses_binned(idx, descs[b].m, p->mode[b])) {
            if (slot_of_group[g] < 0) {
                slot_of_group[g] = (int)p->groups.size();
                FusedGroup fg;
                fg.group = g;
                p->groups.push_back(fg);
            }
            FusedGroup& fg = p->groups[slot_of_group[g]];
            p->fused[b] = slot_of_group[g];
            p->kpl[b] = lj::fused_kpl(idx, p->kpl[b]);
            fg.njobs++;
            fg.keys += descs[b].m;
            p->ws_off[b] = off;
            off = lj::align256(off + lj::fused_job_ws_bytes(descs[b].m, p->kpl[b]));
        } else {
            p->ws_off[b] = off;
            off = lj::align256(off + lj::ws_bytes(idx, descs[b].m, p->mode[b]));
        }
    }
    for (FusedGroup& g : p->groups) {
        g.hdr_off = off;
        off = lj::align256(off + lj::kFusedHeader);
        g.jobs_off = off;
        off = lj::align256(off + (uint64_t)g.njobs * sizeof(lj::FusedJob));
    }
    // Longest-processing-time assignment of the fused launches and the other
    // batches to branches.
    std::vector<uint64_t> load(p->branches, 0);
    p->branch.assign(k, 0);
    for (FusedGroup& g : p->groups) {
        uint32_t r = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        g.branch = r;
        load[r] += g.keys + 1;
    }
    for (uint32_t b : order) {
        if (p->fused[b] >= 0) continue;
        uint32_t r = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        p->branch[b] = r;
        load[r] += descs[b].m + 1;
    }

    hipError_t e = hipMalloc(&p->ws, std::max<uint64_t>(off, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        lj_batch_plan_destroy(p);
        return LJ_ERR_OOM;
    }
    // Job tables of the fused launches.
    for (size_t gi = 0; gi < p->groups.size() && e == hipSuccess; ++gi) {
        FusedGroup& g = p->groups[gi];
        std::vector<lj::FusedJob> jobs;
        uint32_t* hdr = (uint32_t*)((char*)p->ws + g.hdr_off);
        uint32_t tile0 = 0;
        for (uint32_t b : order) {
            if (p->fused[b] != (int)gi) continue;
            const lj_batch_desc& d = descs[b];
            jobs.push_back(lj::make_fused_job(d.index, d.s_keys_dev, d.m, d.out_pairs_dev,
                                              d.out_pairs_dev ? d.out_capacity : 0,
                                              d.out_count_dev, (char*)p->ws + p->ws_off[b],
                                              p->kpl[b], hdr + 1, tile0));
            const uint64_t nt = (uint64_t)tile0 + jobs.back().j.ntiles;
            if (nt >= (1ull << 31)) e = hipErrorInvalidValue;
            tile0 = (uint32_t)nt;
        }
        g.tiles = tile0;
        if (e == hipSuccess)
            e = hipMemcpy((char*)p->ws + g.jobs_off, jobs.data(), jobs.size() * sizeof(jobs[0]),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        lj_batch_plan_destroy(p);
        return LJ_ERR_DEVICE;
    }
    if (p->branches > 1) {
        e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        for (uint32_t r = 0; r < p->branches && e == hipSuccess; ++r) {
            hipStream_t s = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e == hipSuccess) p->streams.push_back(s);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) p->join.push_back(ev);
        }
    }
    if (e == hipSuccess && p->use_graph) {
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) {
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e1 = enqueue_plan(p, cs);
                hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
                e = e1 != hipSuccess ? e1 : e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            (void)hipStreamDestroy(cs);
        }
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        lj_batch_plan_destroy(p);
        return LJ_ERR_DEVICE;
    }
    *out = p;
    return LJ_OK;
}

}  // namespace

extern "C" {

void lj_batch_default_tuning(lj_batch_tuning* tuning) {
    if (tuning) lj::default_tuning(tuning);
}

int lj_batch_plan_create(const lj_batch_desc* descs, uint32_t k, const lj_batch_tuning* tuning,
                         lj_batch_plan** out_plan) {
    try {
        return plan_create(descs, k, tuning, out_plan);
    } catch (const std::bad_alloc&) {
        return LJ_ERR_OOM;
    }
}

int lj_batch_plan_run(lj_batch_plan* p, hipStream_t stream) {
    if (!p) return LJ_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) return LJ_ERR_ARG;
    hipError_t e = p->use_graph ? hipGraphLaunch(p->exec, stream) : enqueue_plan(p, stream);
    return e == hipSuccess ? LJ_OK : LJ_ERR_DEVICE;
}

void lj_batch_plan_destroy(lj_batch_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (hipStream_t s : p->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t ev : p->join) (void)hipEventDestroy(ev);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
}

int lj_batch_autotune(const lj_batch_desc* descs, uint32_t k, hipStream_t stream,
                      lj_batch_tuning* tuning) {
    if (!tuning || !descs) return LJ_ERR_ARG;
    bool present[4] = {false, false, false, false};
    uint64_t max_m = 0;
    for (uint32_t b = 0; b < k; ++b) {
        if (descs[b].m) present[lj::size_class(descs[b].m)] = true;
        max_m = std::max(max_m, descs[b].m);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return LJ_ERR_DEVICE;
    }

    // Mean time of 3 runs after one warm-up (direct launches, no graph).
    auto measure = [&](const lj_batch_tuning& t, int* status) -> float {
        lj_batch_tuning tt = t;
        tt.use_graph = 0;
        lj_batch_plan* p = nullptr;
        *status = lj_batch_plan_create(descs, k, &tt, &p);
        if (*status != LJ_OK) return -1.f;
        float ms = -1.f;
        bool ok = lj_batch_plan_run(p, stream) == LJ_OK &&
                  hipEventRecord(e0, stream) == hipSuccess;
        for (int r = 0; r < 3 && ok; ++r) ok = lj_batch_plan_run(p, stream) == LJ_OK;
        ok = ok && hipEventRecord(e1, stream) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (ok) ms /= 3.f;
        else *status = LJ_ERR_DEVICE;
        (void)hipStreamSynchronize(stream);
        lj_batch_plan_destroy(p);
        return ms;
    };

    lj_batch_tuning best;
    lj::default_tuning(&best);
    int st = LJ_OK;
    float best_ms = measure(best, &st);
    // One kernel per batch instead of the fused launches.
    if (st == LJ_OK) {
        lj_batch_tuning c = best;
        c.fused = 0;
        float ms = measure(c, &st);
        if (st == LJ_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    // Parallel branches, then keys per lane of each size class present.
    for (uint32_t br : {1u, 2u, 8u}) {
        if (st != LJ_OK) break;
        lj_batch_tuning c = best;
        c.branches = br;
        float ms = measure(c, &st);
        if (st == LJ_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    // Binned probe from some batch size on (only sizes some batch reaches).
    for (uint64_t bm : {~0ull, 1ull << 22, 1ull << 20, 1ull << 18}) {
        if (st != LJ_OK) break;
        if (bm != ~0ull && bm > max_m) continue;
        lj_batch_tuning c = best;
        c.binned_min_keys = bm;
        float ms = measure(c, &st);
        if (st == LJ_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    for (int cl = 0; cl < 4 && st == LJ_OK; ++cl) {
        if (!present[cl]) continue;
        for (uint32_t kpl : {4u, 8u, 16u, 24u}) {
            if (kpl == best.keys_per_lane[cl]) continue;
            lj_batch_tuning c = best;
            c.keys_per_lane[cl] = kpl;
            float ms = measure(c, &st);
            if (st != LJ_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LJ_OK) return st;
    best.use_graph = 1;
    best.measured_ms = best_ms;
    *tuning = best;
    return LJ_OK;
}

}  // extern "C"
