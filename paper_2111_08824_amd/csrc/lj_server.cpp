// Serving loop: resident indexes, memory-budget admission, continuous
// batching over several streams, per-request latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lj_batch.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, capacity) with coalescing of freed ranges;
// sizes are multiples of 256 bytes.
class Arena {
   public:
    explicit Arena(uint64_t cap) : cap_(cap) { free_[0] = cap; }
    bool alloc(uint64_t size, uint64_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < size) continue;
            *off = it->first;
            uint64_t rest = it->second - size;
            uint64_t start = it->first + size;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += size;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t size) {
        used_ -= size;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += size;
                return;
            }
        }
        free_[off] = size;
    }
    uint64_t used() const { return used_; }

   private:
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    uint64_t cap_;
    uint64_t used_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    uint32_t index_id = 0;
    bool on_device = false;  // keys and pairs in device memory (no copies)
    int mode = -1;           // probe form (see uses_binned)
    const uint64_t* s_host = nullptr;  // the caller's keys (device memory when on_device)
    uint64_t m = 0;
    lj_pair* out_host = nullptr;  // the caller's pairs (device memory when on_device)
    uint64_t cap = 0;
    uint64_t devcap = 0;  // pairs the device buffer holds
    uint64_t bytes = 0;   // arena footprint
    uint64_t off = 0;     // arena offset
    uint64_t s_off = 0, out_off = 0, ws_off = 0, cnt_off = 0;  // within the block
    bool done = false;
    lj_request_result res{};
};

struct Slot {
    hipStream_t stream = nullptr;      // copies in, probes, counts out
    hipStream_t ret_stream = nullptr;  // pairs back to the host
    std::vector<hipEvent_t> events;    // one per request of a batch
    std::vector<uint32_t> ev_of;       // event that completes each request of the batch
    uint64_t* counts_host = nullptr;   // pinned, one per request of a batch
    uint64_t* counts_dev = nullptr;    // the same memory as the device addresses it
    // Fused launch of the batch's direct probes: job tables staged in pinned
    // memory and copied to fused_dev (launch headers, then the tables).
    lj::FusedJob* jobs_host = nullptr;
    char* fused_dev = nullptr;
    std::vector<Request*> batch;
    bool busy = false;
    bool has_work = false;
    std::condition_variable cv;
    std::thread worker;
};

}  // namespace

struct lj_server {
    int device = -1;
    std::vector<lj_index*> indexes;
    lj_server_config cfg{};
    char* arena_base = nullptr;
    Arena* arena = nullptr;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> requests;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<Slot*> slots;
    std::thread scheduler;
    lj_server_stats stats{};

    void schedule_loop();
    void slot_loop(Slot* s);
    hipError_t enqueue_batch(Slot* s);
    uint32_t grp_tiles_[lj::kFusedGroups] = {};  // scratch of enqueue_batch (scheduler thread)
};

namespace {

// Arena bytes of a request: keys, pairs (host requests only), workspace and
// the count word.
uint64_t footprint(const lj_index* idx, uint64_t m, uint64_t cap, Request* r) {
    const bool dev = r->on_device;
    uint64_t devcap = dev ? cap : std::min<uint64_t>(cap, m * std::max<uint64_t>(idx->max_mult, 1));
    uint64_t off = 0;
    uint64_t s_off = off;
    off = lj::align256(off + (dev ? 0 : 8 * m));
    uint64_t out_off = off;
    off = lj::align256(off + (dev ? 0 : 8 * devcap));
    uint64_t ws_off = off;
    off = lj::align256(off + lj::ws_bytes(idx, m, r->mode));
    uint64_t cnt_off = off;
    off = lj::align256(off + 8);
    if (r) {
        r->devcap = devcap;
        r->s_off = s_off;
        r->out_off = out_off;
        r->ws_off = ws_off;
        r->cnt_off = cnt_off;
        r->bytes = off;
    }
    return off;
}

}  // namespace

// The batch on its slot's stream: the keys of host requests in; one fused
// launch per kernel group for every request probed directly on a plain or
// gapped RMI (their counts written by the kernel straight into the slot's
// pinned count words), followed by one event that completes them all; then
// every other request (binned probes, learned hash indexes, exponential
// search, empty requests) with its own probe, count copy and event, so that
// the completion thread can return each request as soon as its own work is
// done.
hipError_t lj_server::enqueue_batch(Slot* s) {
    hipError_t e = hipSuccess;
    const size_t nb = s->batch.size();
    s->ev_of.assign(nb, 0);
    std::vector<int> grp(nb, -1);
    for (size_t i = 0; i < nb && e == hipSuccess; ++i) {
        Request* r = s->batch[i];
        char* base = arena_base + r->off;
        if (r->m && !r->on_device)  // device requests bring their keys in place
            e = hipMemcpyAsync(base + r->s_off, r->s_host, 8 * r->m, hipMemcpyHostToDevice,
                               s->stream);
        const lj_index* idx = indexes[r->index_id];
        if (cfg.fused && r->m > 0 && !lj::uses_binned(idx, r->m, r->mode))
            grp[i] = lj::fused_group(idx);
    }
    // Fused launches: jobs grouped by kernel group, larger requests first.
    std::vector<uint32_t> order;
    for (size_t i = 0; i < nb; ++i)
        if (grp[i] >= 0) order.push_back((uint32_t)i);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return grp[a] != grp[b] ? grp[a] < grp[b] : s->batch[a]->m > s->batch[b]->m;
    });
    if (!order.empty() && e == hipSuccess) {
        lj::FusedJob* jobs_dev =
            (lj::FusedJob*)(s->fused_dev + lj::kFusedGroups * lj::kFusedHeader);
        size_t a = 0;
        while (a < order.size()) {
            size_t z = a;
            uint32_t tile0 = 0;
            uint32_t* hdr = (uint32_t*)(s->fused_dev + grp[order[a]] * lj::kFusedHeader);
            while (z < order.size() && grp[order[z]] == grp[order[a]]) {
                const uint32_t i = order[z];
                Request* r = s->batch[i];
                char* base = arena_base + r->off;
                const lj_index* idx = indexes[r->index_id];
                lj_pair* out = !r->devcap ? nullptr
                               : r->on_device ? r->out_host
                                              : (lj_pair*)(base + r->out_off);
                s->jobs_host[z] = lj::make_fused_job(
                    idx, r->on_device ? r->s_host : (const uint64_t*)(base + r->s_off), r->m,
                    out, r->devcap, &s->counts_dev[i], base + r->ws_off,
                    cfg.keys_per_lane[lj::size_class(r->m)], hdr + 1, tile0);
                tile0 += s->jobs_host[z].j.ntiles;
                ++z;
            }
            grp_tiles_[grp[order[a]]] = tile0;
            a = z;
        }
        e = hipMemcpyAsync(jobs_dev, s->jobs_host, order.size() * sizeof(lj::FusedJob),
                           hipMemcpyHostToDevice, s->stream);
        a = 0;
        while (a < order.size() && e == hipSuccess) {
            size_t z = a;
            while (z < order.size() && grp[order[z]] == grp[order[a]]) ++z;
            const int g = grp[order[a]];
            e = lj::launch_probe_fused(jobs_dev + a, (uint32_t)(z - a), grp_tiles_[g], g,
                                       (uint32_t*)(s->fused_dev + g * lj::kFusedHeader),
                                       s->stream);
            a = z;
        }
        if (e == hipSuccess) e = hipEventRecord(s->events[order[0]], s->stream);
        for (uint32_t i : order) s->ev_of[i] = order[0];
    }
    for (size_t i = 0; i < nb && e == hipSuccess; ++i) {
        if (grp[i] >= 0) continue;
        Request* r = s->batch[i];
        char* base = arena_base + r->off;
        s->ev_of[i] = (uint32_t)i;
        lj_batch_desc d;
        d.index = indexes[r->index_id];
        d.s_keys_dev = r->on_device ? r->s_host : (const uint64_t*)(base + r->s_off);
        d.m = r->m;
        d.out_pairs_dev = !r->devcap ? nullptr
                          : r->on_device ? r->out_host
                                         : (lj_pair*)(base + r->out_off);
        d.out_capacity = r->devcap;
        d.out_count_dev = (uint64_t*)(base + r->cnt_off);
        if (e == hipSuccess)
            e = lj::enqueue_one(d, base + r->ws_off, cfg.keys_per_lane[lj::size_class(r->m)],
                                r->mode, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&s->counts_host[i], base + r->cnt_off, 8, hipMemcpyDeviceToHost,
                               s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->events[i], s->stream);
    }
    return e;
}

void lj_server::schedule_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        Slot* free_slot = nullptr;
        for (Slot* s : slots)
            if (!s->busy) {
                free_slot = s;
                break;
            }
        if (stopping && queue.empty()) break;
        if (!free_slot || queue.empty()) {
            cv_sched.wait(lk);
            continue;
        }
        // Admit requests in arrival order while the head fits the memory
        // left and the batch limits allow.
        std::vector<Request*> batch;
        uint64_t keys = 0;
        while (!queue.empty() && batch.size() < cfg.max_batch_requests) {
            Request* r = queue.front();
            if (!batch.empty() && keys + r->m > cfg.max_batch_keys) break;
            if (!arena->alloc(r->bytes, &r->off)) break;
            queue.pop_front();
            batch.push_back(r);
            keys += r->m;
        }
        stats.peak_bytes_in_use = std::max(stats.peak_bytes_in_use, arena->used());
        if (batch.empty()) {  // the head waits for memory to be released
            cv_sched.wait(lk);
            continue;
        }
        free_slot->busy = true;
        free_slot->batch = batch;
        stats.batches++;
        stats.max_batch_size = std::max<uint64_t>(stats.max_batch_size, batch.size());
        const uint64_t t = now_ns();
        for (Request* r : batch) {
            r->res.start_ns = t;
            r->res.batch_size = (uint32_t)batch.size();
        }
        lk.unlock();
        hipError_t e = enqueue_batch(free_slot);
        // After a failure part of the batch may already be enqueued: let it
        // finish before the completion thread releases the batch's arena
        // ranges (it skips the per-request waits of failed requests).
        if (e != hipSuccess) (void)hipStreamSynchronize(free_slot->stream);
        lk.lock();
        if (e != hipSuccess) {
            for (Request* r : batch) r->res.status = LJ_ERR_DEVICE;
        }
        free_slot->has_work = true;
        free_slot->cv.notify_one();
    }
}

void lj_server::slot_loop(Slot* s) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        s->cv.wait(lk, [&] { return s->has_work || (stopping && !s->busy); });
        if (!s->has_work) break;
        std::vector<Request*> batch = s->batch;
        lk.unlock();
        // Return requests one by one, as their own work finishes.
        for (size_t i = 0; i < batch.size(); ++i) {
            Request* r = batch[i];
            bool ok = r->res.status == LJ_OK &&
                      hipEventSynchronize(s->events[s->ev_of[i]]) == hipSuccess;
            uint64_t count = ok ? s->counts_host[i] : ~0ull;
            if (ok && count != ~0ull && !r->on_device) {
                uint64_t n = std::min(count, std::min(r->cap, r->devcap));
                if (n)
                    ok = hipMemcpyAsync(r->out_host, arena_base + r->off + r->out_off,
                                        n * sizeof(lj_pair), hipMemcpyDeviceToHost,
                                        s->ret_stream) == hipSuccess &&
                         hipStreamSynchronize(s->ret_stream) == hipSuccess;
            }
            const uint64_t t = now_ns();
            lk.lock();
            if (r->res.status == LJ_OK) {
                if (!ok || count == ~0ull) r->res.status = LJ_ERR_DEVICE;
                else if (count > r->cap) r->res.status = LJ_ERR_CAPACITY;
            }
            r->res.count = count;
            r->res.done_ns = t;
            r->done = true;
            arena->release(r->off, r->bytes);
            stats.requests_done++;
            stats.keys_probed += r->m;
            cv_done.notify_all();
            cv_sched.notify_all();
            lk.unlock();
        }
        (void)hipStreamSynchronize(s->stream);
        lk.lock();
        s->batch.clear();
        s->has_work = false;
        s->busy = false;
        cv_sched.notify_all();
    }
}

extern "C" {

void lj_server_default_config(lj_server_config* c, uint64_t budget_bytes) {
    if (!c) return;
    c->budget_bytes = budget_bytes;
    c->slots = 8;
    c->max_batch_requests = 16;
    c->max_batch_keys = 1ull << 22;
    c->keys_per_lane[0] = 4;
    c->keys_per_lane[1] = 8;
    c->keys_per_lane[2] = 8;
    c->keys_per_lane[3] = 8;
    c->binned_min_keys = 0;
    c->fused = 1;
}

int lj_server_create(lj_index* const* indexes, uint32_t n, const lj_server_config* cfg,
                     lj_server** out) {
    if (!out) return LJ_ERR_ARG;
    *out = nullptr;
    if (!indexes || n == 0 || !cfg || cfg->budget_bytes == 0 || cfg->slots < 1 ||
        cfg->slots > 16 || cfg->max_batch_requests < 1 || cfg->max_batch_keys < 1 ||
        cfg->fused > 1)
        return LJ_ERR_ARG;
    lj_batch_tuning t;
    lj::default_tuning(&t);
    for (int c = 0; c < 4; ++c) t.keys_per_lane[c] = cfg->keys_per_lane[c];
    if (lj::validate_tuning(t) != LJ_OK) return LJ_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LJ_ERR_DEVICE;
    for (uint32_t i = 0; i < n; ++i)
        if (!indexes[i] || indexes[i]->host_only || indexes[i]->device != dev) return LJ_ERR_ARG;

    lj_server* sv = new (std::nothrow) lj_server();
    if (!sv) return LJ_ERR_OOM;
    sv->device = dev;
    sv->indexes.assign(indexes, indexes + n);
    sv->cfg = *cfg;
    sv->cfg.budget_bytes = cfg->budget_bytes & ~255ull;
    int st = LJ_OK;
    if (hipMalloc((void**)&sv->arena_base, sv->cfg.budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        st = LJ_ERR_OOM;
    }
    for (uint32_t i = 0; i < cfg->slots && st == LJ_OK; ++i) {
        Slot* s = new (std::nothrow) Slot();
        if (!s) {
            st = LJ_ERR_OOM;
            break;
        }
        sv->slots.push_back(s);
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&s->ret_stream, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc((void**)&s->counts_host, 8ull * cfg->max_batch_requests) !=
                hipSuccess ||
            hipHostGetDevicePointer((void**)&s->counts_dev, s->counts_host, 0) != hipSuccess ||
            hipHostMalloc((void**)&s->jobs_host,
                          sizeof(lj::FusedJob) * cfg->max_batch_requests) != hipSuccess ||
            hipMalloc((void**)&s->fused_dev, lj::kFusedGroups * lj::kFusedHeader +
                                                 sizeof(lj::FusedJob) * cfg->max_batch_requests) !=
                hipSuccess) {
            (void)hipGetLastError();
            st = LJ_ERR_DEVICE;
            break;
        }
        for (uint32_t q = 0; q < cfg->max_batch_requests && st == LJ_OK; ++q) {
            hipEvent_t ev = nullptr;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
                st = LJ_ERR_DEVICE;
            else
                s->events.push_back(ev);
        }
    }
    if (st != LJ_OK) {
        lj_server_destroy(sv);
        return st;
    }
    sv->arena = new Arena(sv->cfg.budget_bytes);
    for (Slot* s : sv->slots) s->worker = std::thread(&lj_server::slot_loop, sv, s);
    sv->scheduler = std::thread(&lj_server::schedule_loop, sv);
    *out = sv;
    return LJ_OK;
}

}  // extern "C"

namespace {

int submit(lj_server* sv, uint32_t index_id, const uint64_t* s_host, uint64_t m,
           lj_pair* out_host, uint64_t cap, bool on_device, uint64_t* ticket) {
    if (!sv || !ticket || index_id >= sv->indexes.size()) return LJ_ERR_ARG;
    if ((m && !s_host) || (cap && !out_host)) return LJ_ERR_ARG;
    if (m >= (1ull << 32)) return LJ_ERR_TOO_LARGE;
    Request* r = new (std::nothrow) Request();
    if (!r) return LJ_ERR_OOM;
    r->index_id = index_id;
    r->on_device = on_device;
    const uint64_t bmin = sv->cfg.binned_min_keys;
    r->mode = bmin == 0 ? -1 : (m >= bmin ? 1 : 0);
    r->s_host = s_host;
    r->m = m;
    r->out_host = out_host;
    r->cap = out_host ? cap : 0;
    footprint(sv->indexes[index_id], m, r->cap, r);
    if (r->bytes > sv->cfg.budget_bytes) {
        delete r;
        return LJ_ERR_TOO_LARGE;
    }
    r->res.status = LJ_OK;
    r->res.submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) {
        delete r;
        return LJ_ERR_ARG;
    }
    r->ticket = sv->next_ticket++;
    sv->requests[r->ticket] = r;
    sv->queue.push_back(r);
    sv->stats.peak_queue = std::max<uint64_t>(sv->stats.peak_queue, sv->queue.size());
    *ticket = r->ticket;
    sv->cv_sched.notify_all();
    return LJ_OK;
}

}  // namespace

extern "C" {

int lj_server_submit(lj_server* sv, uint32_t index_id, const uint64_t* s_host, uint64_t m,
                     lj_pair* out_host, uint64_t cap, uint64_t* ticket) {
    return submit(sv, index_id, s_host, m, out_host, cap, false, ticket);
}

int lj_server_submit_device(lj_server* sv, uint32_t index_id, const uint64_t* s_dev,
                            uint64_t m, lj_pair* out_dev, uint64_t cap, uint64_t* ticket) {
    return submit(sv, index_id, s_dev, m, out_dev, cap, true, ticket);
}

int lj_server_wait(lj_server* sv, uint64_t ticket, int64_t timeout_ms, lj_request_result* res) {
    if (!sv || !res) return LJ_ERR_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return LJ_ERR_ARG;
    Request* r = it->second;
    if (timeout_ms < 0) {
        sv->cv_done.wait(lk, [&] { return r->done; });
    } else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                     [&] { return r->done; })) {
        return LJ_ERR_TIMEOUT;
    }
    *res = r->res;
    sv->requests.erase(ticket);
    delete r;
    return LJ_OK;
}

int lj_server_replay(lj_server* sv, const lj_replay_request* reqs, uint64_t n,
                     lj_request_result* results) {
    if (!sv || (n && (!reqs || !results))) return LJ_ERR_ARG;
    for (uint64_t i = 1; i < n; ++i)
        if (reqs[i].arrival_ns < reqs[i - 1].arrival_ns) return LJ_ERR_ARG;
    std::vector<uint64_t> tickets;
    try {
        tickets.assign(n, 0);
    } catch (const std::bad_alloc&) {
        return LJ_ERR_OOM;
    }
    std::mutex mu;
    std::condition_variable cv;
    uint64_t submitted = 0;  // requests with a ticket (guarded by mu)
    bool failed = false;
    std::thread collector([&] {
        for (uint64_t i = 0; i < n; ++i) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return submitted > i || failed; });
                if (submitted <= i) return;
            }
            (void)lj_server_wait(sv, tickets[i], -1, &results[i]);
        }
    });
    const uint64_t start = now_ns();
    int st = LJ_OK;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t due = start + reqs[i].arrival_ns;
        for (uint64_t t = now_ns(); t < due; t = now_ns()) {
            if (due - t > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
        }
        uint64_t ticket = 0;
        st = submit(sv, reqs[i].index_id, reqs[i].s_keys_dev, reqs[i].m, reqs[i].out_pairs_dev,
                    reqs[i].out_pairs_dev ? reqs[i].out_capacity : 0, true, &ticket);
        std::lock_guard<std::mutex> lk(mu);
        if (st != LJ_OK) {
            failed = true;
            cv.notify_all();
            break;
        }
        tickets[i] = ticket;
        submitted = i + 1;
        cv.notify_all();
    }
    collector.join();
    return st == LJ_OK ? LJ_OK : LJ_ERR_ARG;
}

int lj_server_get_stats(lj_server* sv, lj_server_stats* out) {
    if (!sv || !out) return LJ_ERR_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    return LJ_OK;
}

void lj_server_destroy(lj_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        sv->cv_sched.notify_all();
        for (Slot* s : sv->slots) s->cv.notify_all();
    }
    if (sv->scheduler.joinable()) sv->scheduler.join();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (Slot* s : sv->slots) s->cv.notify_all();
    }
    for (Slot* s : sv->slots) {
        if (s->worker.joinable()) s->worker.join();
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->ret_stream) (void)hipStreamDestroy(s->ret_stream);
        for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
        if (s->counts_host) (void)hipHostFree(s->counts_host);
        if (s->jobs_host) (void)hipHostFree(s->jobs_host);
        if (s->fused_dev) (void)hipFree(s->fused_dev);
        delete s;
    }
    for (auto& kv : sv->requests) delete kv.second;
    if (sv->arena_base) (void)hipFree(sv->arena_base);
    delete sv->arena;
    delete sv;
}

}  // extern "C"
