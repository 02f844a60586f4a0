/*
 * lj.h -- learned indexed nested loop join on MI355X (gfx950).
 *
 * The operation (Section II-A, "Indexed Nested Loop Joins"; Section III,
 * "Learned Indexed Nested Loop Join"): the inner relation R is indexed by a
 * two-level linear RMI (Section II-D, "Recursive Model Index"): a root model
 * picks a leaf model, the leaf model predicts a position, and the leaf's
 * min/max error bounds limit a last-mile search.  Each key of the outer
 * relation S probes the index and every tuple of R with the same key is a
 * match; duplicates are found by scanning the bounded range around the
 * prediction (Section VI-B, "Duplicates").  The result is the set of pairs
 *
 *     { (s_idx, r_idx) : S[s_idx] == R[r_idx] }
 *
 * emitted in ascending (s_idx, r_idx) order, where r_idx is the position in
 * the sorted R and s_idx the position in S as passed.  Two more index kinds
 * are built over the same RMI and give the same pairs: the gapped RMI
 * (Section III-A) and the learned hash index (Section III-C).
 *
 * Conventions for every entry point:
 *   - Status codes are returned; nothing throws across this interface.
 *   - Keys are uint64.  n (|R|) must be below 2^31 and m (|S|) below 2^32.
 *   - "_dev" pointers are device memory of the index's GPU; "_host" pointers
 *     are host memory.  Caller-owned buffers stay caller-owned.
 *   - An index is immutable after lj_build_rmi: concurrent probes of one
 *     index from several host threads or streams are safe.
 *   - Work is enqueued on `stream` (0 = the null stream) of the index's
 *     device; calls fail with LJ_ERR_ARG if another device is current.
 */
#ifndef LJ_H
#define LJ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lj_index lj_index; /* opaque, library-owned */

/* One output pair (8 bytes). */
typedef struct {
    uint32_t s_idx;
    uint32_t r_idx;
} lj_pair;

enum {
    LJ_OK = 0,
    LJ_ERR_ARG = -1,       /* null pointer, zero leaves, bad flags, wrong device */
    LJ_ERR_UNSORTED = -2,  /* R is not non-decreasing */
    LJ_ERR_TOO_LARGE = -3, /* n >= 2^31, m >= 2^32 or leaves > 2^26 */
    LJ_ERR_CAPACITY = -4,  /* more pairs than out_capacity (count still set) */
    LJ_ERR_DEVICE = -5,    /* a HIP call failed, or a kernel reported an error */
    LJ_ERR_OOM = -6,       /* device or host allocation failed */
    LJ_ERR_WORKSPACE = -7, /* workspace smaller than lj_probe_workspace_bytes() */
    LJ_ERR_TIMEOUT = -8    /* a wait ended before the request completed */
};

/* Build flags.  Exactly one leaf arithmetic must be given to lj_build_rmi;
 * the search flag is optional. */
enum {
    LJ_LEAF_FP32 = 1u,          /* leaf model evaluated with fmaf on f32 parameters */
    LJ_LEAF_FP64 = 2u,          /* leaf model evaluated with fma on f64 parameters */
    LJ_SEARCH_EXPONENTIAL = 4u, /* last-mile search gallops out from the prediction
                                   (steps 8, 16, 32, ...) inside the error bounds, then
                                   bisects; without it, binary search over the bounds */
    LJ_PROBE_BINNED = 8u,       /* probes put S in key order first: 4096 equi-depth key
                                   ranges of R, two stable partition passes, searches
                                   in that order with each XCD on its own ranges, results
                                   put back in S order before emission (the locality of
                                   buffering requests per node, Section III-B).  Same
                                   output; about 28 more workspace bytes per outer key */
    LJ_ROOT_RADIX = 16u         /* root model = piecewise-linear CDF over a radix table
                                   of the key instead of one least-squares line (the
                                   radix-table idea of RadixSpline, Section II-D; the
                                   paper's RMIs are tuned over root model types).  The
                                   key's offset from R[0] picks one of 3776 buckets by
                                   its exponent and next 6 bits; the table holds the
                                   leaf coordinate leaves * rank / n of every bucket
                                   edge and the root interpolates inside the bucket in
                                   integer arithmetic.  Leaves then hold about n / leaves
                                   keys each on skewed data too (a line puts most keys
                                   of a heavy-tailed R into a few leaves).  Same output;
                                   15 KB more per index */
};

/*
 * Build the two-level linear RMI over R (Section II-D; building happens
 * offline and is not part of the join, Section III-A, "GRMI Building").
 *
 *   r_keys_host  n keys in host memory, non-decreasing (duplicates allowed).
 *                Read only during the call; the index keeps its own device
 *                copy of R.
 *   n            number of keys, 0 <= n < 2^31.  n = 0 gives an index for
 *                which every probe finds nothing.
 *   leaves       number of leaf models, 1 <= leaves <= 2^26.
 *   flags        LJ_LEAF_FP32 or LJ_LEAF_FP64, optionally with
 *                LJ_SEARCH_EXPONENTIAL and LJ_PROBE_BINNED (the result is
 *                the same; only the order of the work changes).
 *   stream       stream used for the uploads (the call returns after they
 *                complete).
 *   out_index    receives the new index; free it with lj_free_index.
 *
 * The index also keeps the first key of every 16-key (128-byte) line of R:
 * the binary search first bisects these line samples inside the window,
 * then the candidate positions of one line of R.
 *
 * Fitting: the root is an FP64 least-squares line from (key - R[0]) to
 * leaf coordinate i*leaves/n; each leaf is an FP64 least-squares line from
 * (key - first key of the leaf) to the offset inside the leaf, rounded to
 * f32 for LJ_LEAF_FP32.  The per-leaf min/max error bounds are then
 * recomputed for every key of R under exactly the arithmetic the probe uses
 * (f32 or f64), so the search window of any key of R holds all its copies.
 *
 * Errors: LJ_ERR_ARG, LJ_ERR_UNSORTED, LJ_ERR_TOO_LARGE, LJ_ERR_OOM,
 * LJ_ERR_DEVICE.  On error *out_index is set to NULL.
 */
int lj_build_rmi(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                 uint32_t flags, hipStream_t stream, lj_index** out_index);

/*
 * Build a gapped RMI (Section III-A, "Gapped RMI"): the same two-level RMI,
 * then model-based insertion of R, in order, into gapped arrays of
 * slots_per_key * n slots (a little more when predictions run past the
 * end): key i goes to its predicted slot, or, when that slot is taken, to
 * the slot right after key i - 1.  Keys, their payloads (the position in R)
 * and the gap bitmap share one 16-byte slot; a gap holds the next key of R.
 * A probe predicts the slot and searches exponentially forward from it
 * (Section III-A, "GRMI Lookup"), bounded by the leaf's largest insertion
 * drift; every entry point that takes an index (probes, plans, the server,
 * LJ_PROBE_BINNED) works on it and emits the same pairs as for a plain RMI.
 *
 *   slots_per_key  1..16; the evaluation's setting of 4 gaps per key is
 *                  read as 4 slots per key (the hash baselines matched to
 *                  it run at load factor 25%).  Device memory: 16 bytes per
 *                  slot, on top of R and the leaf table.
 *
 * Other arguments and errors as lj_build_rmi; LJ_ERR_ARG also for
 * slots_per_key outside 1..16; LJ_ERR_TOO_LARGE also when the slot count
 * reaches 2^32.
 */
int lj_build_gapped_rmi(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                        uint32_t slots_per_key, uint32_t flags, hipStream_t stream,
                        lj_index** out_index);

/*
 * Build a learned hash index (Section III-C, "Learned-based Hash INLJ"):
 * the same two-level RMI serves as an order-preserving hash function into a
 * bucket-chained table; nothing is searched.  The bucket of a key is its
 * predicted position in R (clamped into its leaf's run) times
 * slots_per_key / 4, so there are about slots_per_key * n / 4 primary
 * buckets of 4 slots (64 bytes: 4 keys, their positions in R, the next
 * bucket of the chain, the number of keys held).  Keys of R are appended to
 * their chain in R order, so all copies of a key share one chain, in
 * order.  A probe walks the chain of its key's bucket; every entry point
 * that takes an index works on it and emits the same pairs as for a plain
 * RMI.
 *
 *   slots_per_key  1..16 (4: one bucket of 4 slots per key of R, the
 *                  bucket size and load factor of the evaluation's hash
 *                  baseline).  Device memory: 64 bytes per bucket,
 *                  overflow buckets included, on top of R and the leaves.
 *
 * Other arguments and errors as lj_build_gapped_rmi.
 */
int lj_build_learned_hash(const uint64_t* r_keys_host, uint64_t n, uint32_t leaves,
                          uint32_t slots_per_key, uint32_t flags, hipStream_t stream,
                          lj_index** out_index);

/* Release an index and its device memory.  NULL is ignored.  The caller
 * must ensure no probe of this index is still running on any stream. */
void lj_free_index(lj_index* index);

/*
 * Probe the index with every key of S and emit the matching pairs
 * (Section II-A; Section III).  Synchronous in the count: the call returns
 * after the probe has finished on `stream`.
 *
 *   s_keys_dev     m outer keys in device memory (any alignment of 8).
 *   m              number of outer keys, 0 <= m < 2^32.
 *   out_pairs_dev  room for out_capacity pairs, or NULL with out_capacity
 *                  0 for a count-only probe (which returns LJ_OK).
 *   out_count_host receives the total number of matching pairs.
 *
 * Capacity protocol (like snprintf): the pairs whose rank in the output
 * order is below out_capacity are written; *out_count_host is always the
 * true total; if it exceeds out_capacity the call returns LJ_ERR_CAPACITY
 * and the caller may retry with a larger buffer.
 *
 * Scratch memory is taken from a per-stream cache owned by the library
 * (grown with hipMalloc when too small).  Errors: LJ_ERR_ARG,
 * LJ_ERR_TOO_LARGE, LJ_ERR_CAPACITY, LJ_ERR_DEVICE, LJ_ERR_OOM.
 */
int lj_probe_join(const lj_index* index, const uint64_t* s_keys_dev, uint64_t m,
                  lj_pair* out_pairs_dev, uint64_t out_capacity,
                  uint64_t* out_count_host, hipStream_t stream);

/* Bytes of device workspace lj_probe_join_async needs for m outer keys
 * against `index` (0 for a NULL index). */
uint64_t lj_probe_workspace_bytes(const lj_index* index, uint64_t m);

/*
 * Asynchronous probe: same result as lj_probe_join, but nothing is read
 * back and nothing is allocated, so the call can be captured in a HIP graph.
 *
 *   out_count_dev   device uint64 that receives the total pair count, or
 *                   UINT64_MAX if a kernel hit its internal wait bound (a
 *                   device fault condition; the pairs are then invalid).
 *   workspace_dev   caller-owned device scratch of at least
 *                   lj_probe_workspace_bytes(index, m) bytes, 256-byte aligned;
 *                   calls that share one workspace must be ordered on one
 *                   stream.
 *
 * The capacity protocol is the same; the caller compares *out_count_dev
 * with out_capacity after the stream completes.
 * Errors (host-side checks only): LJ_ERR_ARG, LJ_ERR_TOO_LARGE,
 * LJ_ERR_WORKSPACE, LJ_ERR_DEVICE (launch failure).
 */
int lj_probe_join_async(const lj_index* index, const uint64_t* s_keys_dev,
                        uint64_t m, lj_pair* out_pairs_dev,
                        uint64_t out_capacity, uint64_t* out_count_dev,
                        void* workspace_dev, uint64_t workspace_bytes,
                        hipStream_t stream);

/*
 * Probe that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the result and capacity protocol of
 * lj_probe_join_async, always by the direct probe, with the probe's
 * workspace (tile and done counters, error flag, one status word per tile)
 * in a fixed 4 MiB device array that the library holds on every GPU it runs
 * on until the process ends.  No hipMalloc, hipFree or other allocation is
 * made; the array is cleared by a kernel at the start of every call.
 *
 *   m              0 <= m <= lj_probe_join_noalloc_max_keys() (536,838,144);
 *                  larger m returns LJ_ERR_TOO_LARGE.
 *   out_count_dev  device uint64 receiving the total pair count (UINT64_MAX
 *                  if a kernel hit its internal wait bound).
 *
 * All calls on one GPU share that GPU's array: calls that overlap on one
 * GPU (two streams, or two host threads) race and give wrong results; order
 * them on one stream.  Errors (host-side checks only): LJ_ERR_ARG,
 * LJ_ERR_TOO_LARGE, LJ_ERR_DEVICE.
 */
uint64_t lj_probe_join_noalloc_max_keys(void);
int lj_probe_join_noalloc(const lj_index* index, const uint64_t* s_keys_dev, uint64_t m,
                          lj_pair* out_pairs_dev, uint64_t out_capacity,
                          uint64_t* out_count_dev, hipStream_t stream);

/*
 * Batched probe of many indexes as one replayable unit.
 *
 * Each descriptor is one independent probe with the semantics and capacity
 * protocol of lj_probe_join_async: the keys of s_keys_dev against `index`,
 * pairs into out_pairs_dev, the total into *out_count_dev.  A plan fixes the
 * descriptors, owns the device workspace, spreads the batches over parallel
 * branches (streams forked from and joined back into the caller's stream,
 * largest batches first, each branch taking the next batch while it has the
 * least work) and captures the whole fork/join of fused probe kernels once
 * into a HIP graph; running the plan replays the graph with no host work,
 * so new key values in the same buffers are probed at the cost of one
 * graph launch.
 */
typedef struct {
    const lj_index* index;
    const uint64_t* s_keys_dev;
    uint64_t m;
    lj_pair* out_pairs_dev;   /* NULL with out_capacity 0 for count only */
    uint64_t out_capacity;
    uint64_t* out_count_dev;  /* receives the total (UINT64_MAX on device error) */
} lj_batch_desc;

/*
 * Launch shape of a plan.  Batches fall in four size classes
 * (m < 2^13, < 2^17, < 2^21, larger); a class's tiles hold
 * 256 * keys_per_lane[class] outer keys, with keys_per_lane in
 * {4, 8, 16, 24} (24 is lowered to 16 for indexes with duplicate keys);
 * the default is {4, 8, 8, 8}.
 * `branches` (1..16) is the number of parallel streams the batches are
 * spread over; `use_graph` selects graph replay (1) or direct launches (0).
 * `binned_min_keys`: batches of at least this many outer keys use the
 * binned probe (LJ_PROBE_BINNED) and smaller ones the direct probe; 0 keeps
 * each index's own choice, UINT64_MAX probes every batch directly.
 * `fused` = 1: all batches probed directly on plain RMIs (binary search) or
 * gapped RMIs run in one kernel per index kind, leaf arithmetic and
 * duplicate class (usually one launch for the whole plan): the tiles of
 * every batch share one tile-id queue, each tile with its own batch's keys
 * per lane (4 or 8: larger settings run as 8); 0: one kernel per batch.  `measured_ms` is filled by lj_batch_autotune.
 */
typedef struct {
    uint32_t keys_per_lane[4];
    uint32_t branches;
    uint32_t use_graph;
    uint64_t binned_min_keys;
    float measured_ms;
    uint32_t fused;
} lj_batch_tuning;

typedef struct lj_batch_plan lj_batch_plan;

/* Fill *tuning with the built-in default launch shape. */
void lj_batch_default_tuning(lj_batch_tuning* tuning);

/*
 * Create a plan for k descriptors (k >= 1; copied, so the array may be
 * freed).  tuning may be NULL for the default.  The indexes and buffers
 * named by the descriptors must outlive the plan.  Synchronous.
 * Errors: LJ_ERR_ARG (null pointer, host-only index, wrong device, bad
 * tuning), LJ_ERR_TOO_LARGE (m >= 2^32), LJ_ERR_OOM, LJ_ERR_DEVICE.
 */
int lj_batch_plan_create(const lj_batch_desc* descs, uint32_t k,
                         const lj_batch_tuning* tuning, lj_batch_plan** out_plan);

/* Enqueue one run of the plan on `stream` (asynchronous; the run is ordered
 * after earlier work on `stream` and later work waits for it).  Runs of one
 * plan must not overlap: they share its workspace.  Errors: LJ_ERR_ARG,
 * LJ_ERR_DEVICE. */
int lj_batch_plan_run(lj_batch_plan* plan, hipStream_t stream);

/* Free a plan (after its runs have completed).  NULL is ignored. */
void lj_batch_plan_destroy(lj_batch_plan* plan);

/*
 * Autotuner: times candidate launch shapes (branch counts, the batch size
 * from which the binned probe is used, and keys per lane for each size
 * class present) on the device with these descriptors,
 * by coordinate descent from the default, and returns the fastest in
 * *tuning (measured_ms = its mean time per run).  Runs the probes several
 * times, writing the descriptors' outputs.  Synchronous.  Errors as for
 * lj_batch_plan_create.
 */
int lj_batch_autotune(const lj_batch_desc* descs, uint32_t k, hipStream_t stream,
                      lj_batch_tuning* tuning);

/*
 * Serving loop: several indexes resident in HBM, probe requests admitted by
 * memory and batched continuously.
 *
 * Requests carry host buffers: the server copies the outer keys to the
 * device, probes, and copies the pairs back.  A scheduler thread admits
 * requests in arrival order while the head request's device footprint
 * (keys + output + workspace) fits the memory budget left, forms a batch as
 * soon as one of `slots` streams is free (so requests that arrive while
 * others run join the next batch), and enqueues the batch on that stream:
 * the key copies, then (with `fused`) one kernel per kernel group for all
 * requests probed directly on plain or gapped RMIs, which writes each
 * request's count straight into pinned host memory, then every other
 * request's probe and count copy; batches on different streams overlap on
 * the device and on the copy engines.  A completion thread per stream
 * returns each request as soon as its work is done (pairs copied back on a
 * second stream), frees its memory and wakes its waiter.  Device memory
 * for requests comes from one arena of `budget_bytes` allocated at
 * creation.
 */
typedef struct {
    uint64_t budget_bytes;        /* device memory for request buffers (> 0) */
    uint32_t slots;               /* batches in flight, 1..16 */
    uint32_t max_batch_requests;  /* requests per batch, >= 1 */
    uint64_t max_batch_keys;      /* outer keys per batch (a larger single request
                                     still forms a batch alone), >= 1 */
    uint32_t keys_per_lane[4];    /* tile shape per size class, as in lj_batch_tuning */
    uint64_t binned_min_keys;     /* requests of at least this many keys use the binned
                                     probe, smaller ones the direct probe; 0 keeps each
                                     index's own choice (LJ_PROBE_BINNED) */
    uint32_t fused;               /* 1: a batch's direct probes on plain or gapped RMIs
                                     run in one fused launch (see lj_batch_tuning);
                                     0: one probe kernel and count copy per request */
    uint32_t pad;
} lj_server_config;

typedef struct lj_server lj_server;

typedef struct {
    int32_t status;        /* LJ_OK, LJ_ERR_CAPACITY (pairs truncated) or an error */
    uint32_t batch_size;   /* requests in the batch this request ran in */
    uint64_t count;        /* total matching pairs */
    uint64_t submit_ns;    /* steady-clock times of submission, launch, completion */
    uint64_t start_ns;
    uint64_t done_ns;
} lj_request_result;

typedef struct {
    uint64_t requests_done;
    uint64_t batches;
    uint64_t peak_bytes_in_use;   /* never above budget_bytes */
    uint64_t peak_queue;          /* requests waiting for admission */
    uint64_t max_batch_size;
    uint64_t keys_probed;
} lj_server_stats;

/* Fill *config with defaults for a budget: 8 slots, 16 requests and 2^22
 * keys per batch, keys per lane 4/8/8/8, binned_min_keys 0, fused 1. */
void lj_server_default_config(lj_server_config* config, uint64_t budget_bytes);

/*
 * Start a server over `n_indexes` indexes (not owned; they must outlive
 * the server and live on the current device).  Allocates the arena and
 * starts the threads.  Errors: LJ_ERR_ARG, LJ_ERR_OOM, LJ_ERR_DEVICE.
 */
int lj_server_create(lj_index* const* indexes, uint32_t n_indexes,
                     const lj_server_config* config, lj_server** out_server);

/*
 * Submit a request: probe index `index_id` with the m keys at s_keys_host;
 * up to out_capacity pairs go to out_pairs_host.  Both host buffers must
 * stay valid until the request completes (pinned memory makes the copies
 * asynchronous).  Returns at once with a ticket.  Errors: LJ_ERR_ARG,
 * LJ_ERR_TOO_LARGE (m >= 2^32, or the request alone exceeds the budget:
 * it could never be admitted).
 */
int lj_server_submit(lj_server* server, uint32_t index_id, const uint64_t* s_keys_host,
                     uint64_t m, lj_pair* out_pairs_host, uint64_t out_capacity,
                     uint64_t* out_ticket);

/*
 * Submit a request whose keys and pairs already live in device memory of
 * the server's GPU (for producers and consumers on the GPU): no copies are
 * made; the probe reads s_keys_dev and writes up to out_capacity pairs to
 * out_pairs_dev directly, and only its workspace and count word come from
 * the arena.  The server's streams do not wait for the caller's: the work
 * that writes the keys (or last uses the pair buffer) must be complete when
 * this is called.  Both buffers must stay valid and untouched until the
 * request completes.  Same tickets, results and errors as lj_server_submit.
 */
int lj_server_submit_device(lj_server* server, uint32_t index_id,
                            const uint64_t* s_keys_dev, uint64_t m,
                            lj_pair* out_pairs_dev, uint64_t out_capacity,
                            uint64_t* out_ticket);

/*
 * Wait until a request completes (timeout_ms < 0: no limit) and fetch its
 * result; a ticket can be waited for once.  Returns LJ_OK when the result
 * was fetched (the request's own status is in result->status),
 * LJ_ERR_TIMEOUT if it did not complete in time, LJ_ERR_ARG for an
 * unknown ticket.
 */
int lj_server_wait(lj_server* server, uint64_t ticket, int64_t timeout_ms,
                   lj_request_result* result);

/*
 * Load driver for device-resident requests (measurement of the serving loop
 * without a client's own per-request cost): the calling thread submits the
 * n requests with lj_server_submit_device, each at its arrival time
 * (arrival_ns after the call starts, non-decreasing; 0 for all at once),
 * while a second thread waits for them in submission order; returns when
 * every request has completed, with request i's result in results[i] (its
 * own status inside).  Errors: LJ_ERR_ARG (null pointers, decreasing
 * arrival times, or a submission refused: results of the requests before it
 * are valid), LJ_ERR_OOM.
 */
typedef struct {
    uint32_t index_id;
    uint32_t pad;
    const uint64_t* s_keys_dev;
    uint64_t m;
    lj_pair* out_pairs_dev;   /* NULL with out_capacity 0 for count only */
    uint64_t out_capacity;
    uint64_t arrival_ns;
} lj_replay_request;

int lj_server_replay(lj_server* server, const lj_replay_request* requests, uint64_t n,
                     lj_request_result* results);

int lj_server_get_stats(lj_server* server, lj_server_stats* out);

/* Finish every submitted request, stop the threads and free the arena. */
void lj_server_destroy(lj_server* server);

/* Summary of an index (sizes and model quality). */
typedef struct {
    uint64_t n;               /* keys in R */
    uint32_t leaves;          /* leaf models */
    uint32_t flags;           /* the build flags */
    uint32_t nonempty_leaves; /* leaves with at least one key */
    uint32_t max_leaf_keys;   /* keys in the largest leaf */
    uint64_t max_mult;        /* longest run of equal keys in R */
    double mean_window;       /* mean search-window length over the keys of R
                                 (in slots for a gapped RMI; for a learned
                                 hash, the mean number of buckets a probe of
                                 a key of R reads) */
    uint64_t max_window;      /* largest search window of any leaf */
    uint64_t device_bytes;    /* device memory held (R, line samples, leaves,
                                 fences, and the slot or bucket arrays) */
    double root_a0, root_b0;  /* root model parameters */
    uint64_t root_kmin;       /* root model key origin (R[0]) */
    uint32_t slots_per_key;   /* gapped RMI or learned hash: slots per key of R
                                 (0: plain RMI) */
    uint32_t pad;
    uint64_t nslots;          /* gapped RMI: slots of the gapped arrays;
                                 learned hash: 4 per bucket, overflow included */
} lj_index_stats;

int lj_index_get_stats(const lj_index* index, lj_index_stats* out);

/*
 * Device self-check: a GPU kernel routes and predicts every key of R with
 * the device arithmetic and counts keys whose own position falls outside
 * their search window (0 means the host-built bounds hold on the device);
 * for a gapped RMI, every key slot whose key differs from R at its payload
 * position or lies outside its slot window, plus the difference between
 * the number of key slots and n; for a learned hash, every key of R not
 * found in the chain of its bucket, plus the difference between the number
 * of keys the buckets hold and n.
 * Synchronous.  Errors: LJ_ERR_ARG, LJ_ERR_DEVICE, LJ_ERR_OOM.
 */
int lj_self_check(const lj_index* index, uint64_t* out_violations_host,
                  hipStream_t stream);

/*
 * Window diagnostics: for each of m keys (device memory), the leaf chosen by
 * the root, the predicted absolute position (-1 for an empty leaf) and the
 * absolute search window [lo, hi] the probe searches (lo > hi = empty
 * window); for a gapped RMI the predicted slot and the slot window; for a
 * learned hash the primary bucket (pred = lo = hi).  Used by tests and for
 * model-quality statistics; not part of the
 * join.  Any output pointer may be NULL.  Asynchronous on `stream`.
 */
int lj_predict_windows(const lj_index* index, const uint64_t* keys_dev,
                       uint64_t m, uint32_t* leaf_dev, int64_t* pred_dev,
                       int64_t* win_lo_dev, int64_t* win_hi_dev,
                       hipStream_t stream);

/*
 * Host-side model evaluation for tests without a GPU: the same leaf choice,
 * prediction and window as lj_predict_windows, computed on the CPU from an
 * index's host copy of the model.
 */
int lj_predict_windows_host(const lj_index* index, const uint64_t* keys_host,
                            uint64_t m, uint32_t* leaf_host,
                            int64_t* pred_host, int64_t* win_lo_host,
                            int64_t* win_hi_host);

/*
 * Build only the host-side model (no device allocation) so that the fit and
 * its bounds can be tested without a GPU.  The index can be queried with
 * lj_index_get_stats and lj_predict_windows_host; probing it returns
 * LJ_ERR_ARG.  Same arguments and errors as lj_build_rmi.
 */
int lj_build_rmi_host_only(const uint64_t* r_keys_host, uint64_t n,
                           uint32_t leaves, uint32_t flags,
                           lj_index** out_index);

/* Host-only build of a gapped RMI (arguments as lj_build_gapped_rmi); its
 * slot arrays can be read with lj_gapped_slots_host. */
int lj_build_gapped_rmi_host_only(const uint64_t* r_keys_host, uint64_t n,
                                  uint32_t leaves, uint32_t slots_per_key,
                                  uint32_t flags, lj_index** out_index);

/*
 * Copy the slot arrays of a host-only gapped RMI: for slot j < capacity,
 * keys_host[j] (the key, or for a gap the next key of R) and ridx_host[j]
 * (the key's position in R, or UINT32_MAX for a gap); *nslots_out receives
 * the number of slots.  Errors: LJ_ERR_ARG (not a host-only gapped index),
 * LJ_ERR_CAPACITY (capacity below the slot count; the first slots are
 * copied).
 */
int lj_gapped_slots_host(const lj_index* index, uint64_t* keys_host,
                         uint32_t* ridx_host, uint64_t capacity,
                         uint64_t* nslots_out);

/* Host-only build of a learned hash index (arguments as
 * lj_build_learned_hash); its buckets can be read with lj_hash_buckets_host. */
int lj_build_learned_hash_host_only(const uint64_t* r_keys_host, uint64_t n,
                                    uint32_t leaves, uint32_t slots_per_key,
                                    uint32_t flags, lj_index** out_index);

/*
 * Copy the buckets of a host-only learned hash index: for bucket b <
 * capacity, keys_host[4b + j] and ridx_host[4b + j] for its slots j < 4
 * (key 0 and UINT32_MAX for an empty slot) and next_host[b] (the next
 * bucket of the chain, UINT32_MAX at the end).  Buckets [0, *nprimary_out)
 * are the primary ones; *nbuckets_out receives the number of buckets.
 * nprimary_out may be NULL.  Errors: LJ_ERR_ARG (not a host-only learned
 * hash index), LJ_ERR_CAPACITY (capacity below the bucket count; the first
 * buckets are copied).
 */
int lj_hash_buckets_host(const lj_index* index, uint64_t* keys_host,
                         uint32_t* ridx_host, uint32_t* next_host,
                         uint64_t capacity, uint64_t* nbuckets_out,
                         uint64_t* nprimary_out);

/*
 * Learned sort join (Section IV): the join of two relations in any order,
 *
 *     { (s_idx, r_idx) : S[s_idx] == R[r_idx] }
 *
 * in ascending (s_idx, r_idx) order, with r_idx and s_idx the positions in
 * R and S as passed (no index is built beforehand).  The phases follow
 * Section IV-B..D: a CDF model of R from a sorted sample (a linear spline
 * over equi-depth sample knots), range partitioning of R by the model
 * scaled up (histograms, prefix sums, stable scatter passes), a bitonic
 * sort of each partition (Section IV-C), and a join in which each key of S
 * is looked up in the one partition of the sorted R its key maps to
 * (Section IV-D).  Asynchronous; nothing is allocated, so calls can be
 * captured in a HIP graph.
 *
 *   r_keys_dev    n keys of R in device memory, n < 2^31.
 *   s_keys_dev    m keys of S in device memory, m < 2^32.
 *   out_pairs_dev room for out_capacity pairs, or NULL with capacity 0
 *                 (count only).  Capacity protocol of lj_probe_join_async.
 *   out_count_dev device uint64 receiving the total pair count, or
 *                 UINT64_MAX if a kernel hit its internal wait bound.
 *   workspace_dev caller-owned device scratch of at least
 *                 lj_sort_join_workspace_bytes(n, m) bytes (about
 *                 33 n + 32 m bytes), 256-byte aligned; calls sharing one
 *                 workspace must be ordered on one stream.
 *
 * The benchmark timing hook (lj_probe_set_timing_events) brackets the join
 * kernel over the partitioned S.  Errors (host-side checks only):
 * LJ_ERR_ARG, LJ_ERR_TOO_LARGE, LJ_ERR_WORKSPACE, LJ_ERR_DEVICE.
 */
uint64_t lj_sort_join_workspace_bytes(uint64_t n, uint64_t m);
int lj_sort_join_async(const uint64_t* r_keys_dev, uint64_t n,
                       const uint64_t* s_keys_dev, uint64_t m,
                       lj_pair* out_pairs_dev, uint64_t out_capacity,
                       uint64_t* out_count_dev, void* workspace_dev,
                       uint64_t workspace_bytes, hipStream_t stream);

/*
 * The sort phase of the learned sort join on its own (Section IV-B and
 * IV-C): keys_dev (n keys, any order) into sorted_keys_dev and, for each
 * output slot, the input position of its key in positions_dev, in
 * ascending (key, position) order.  Workspace: at least
 * lj_sort_join_workspace_bytes(n, 0) bytes, 256-byte aligned.  Output
 * buffers are caller-owned and must not overlap keys_dev.  Asynchronous.
 * Errors: LJ_ERR_ARG, LJ_ERR_TOO_LARGE (n >= 2^31), LJ_ERR_WORKSPACE,
 * LJ_ERR_DEVICE.
 */
int lj_learned_sort_async(const uint64_t* keys_dev, uint64_t n,
                          uint64_t* sorted_keys_dev, uint32_t* positions_dev,
                          void* workspace_dev, uint64_t workspace_bytes,
                          hipStream_t stream);

/*
 * Timing hook for benchmarks: the next lj_probe_join, lj_probe_join_async or
 * lj_sort_join_async call made by this host thread records `start`
 * immediately before and `stop` immediately after its probe kernel (with
 * LJ_PROBE_BINNED: the search kernel over the partitioned keys; for the
 * sort join: its join kernel), on the call's stream.  Pass
 * NULL events to disable.
 */
int lj_probe_set_timing_events(hipEvent_t start, hipEvent_t stop);

/*
 * Random-access ceiling for the roofline: reads `reads` 8-byte words, each
 * from a pseudo-random `granule`-byte aligned block of the device buffer
 * `buf_dev` (`bytes` long), with every lane keeping 8 independent loads in
 * flight; a checksum goes to `sink_dev` (one u64) so no load is elided.
 * Asynchronous on `stream`; time it with events.  `granule` is a power of
 * two in [8, 4096] and `bytes` at least `granule`.  Errors: LJ_ERR_ARG,
 * LJ_ERR_DEVICE.
 */
int lj_bench_random_gather(const void* buf_dev, uint64_t bytes,
                           uint32_t granule, uint64_t reads, uint64_t seed,
                           uint64_t* sink_dev, hipStream_t stream);

/* Static description of a status code. */
const char* lj_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* LJ_H */
