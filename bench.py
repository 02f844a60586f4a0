#!/usr/bin/env python3
"""Benchmark of the learned indexed nested loop join probe on one MI355X.

One step = one synchronous probe (lj_probe_join) of the whole outer relation
S against the two-level RMI over R: root model, linear leaf model, bounded
last-mile search, match counting, output compaction and pair emission, plus
the 8-byte count readback.  R, the index and S are resident in HBM before
the timed region; building the index is offline (untimed).  By default the
probe is the binned one (S partitioned by key range of R first, the same
pairs in the same order); --probe direct probes S in its own order.  The
root is the radix-table root by default (--root linear: one least-squares
line).

Default workload: R = 2e8 distinct lognormal(0, 2) keys scaled to 2^63,
2^20 leaves with FP32 leaf models; S = 2e8 keys, 90% Zipf(1) hits.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: the
build targets one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "outer-key probes/sec + achieved HBM GB/s vs roofline; p50/p99 probe latency"
HBM_PEAK_GBS = 8000.0
PROBE_KERNEL_SOURCES = ["paper_2111_08824_amd/csrc/lj_kernels.hip",
                        "paper_2111_08824_amd/csrc/lj_partition.hip",
                        "paper_2111_08824_amd/csrc/lj_device.h",
                        "paper_2111_08824_amd/csrc/rmi_eval.h",
                        "paper_2111_08824_amd/csrc/lj_internal.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in PROBE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SORT_JOIN_SOURCES = ["paper_2111_08824_amd/csrc/lj_sortjoin.hip",
                     "paper_2111_08824_amd/csrc/lj_sortjoin.h",
                     "paper_2111_08824_amd/csrc/lj_device.h",
                     "paper_2111_08824_amd/csrc/lj_internal.h"]


def kernel_source_hash_sort_join() -> str:
    h = hashlib.sha256()
    for f in SORT_JOIN_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_summary(path: str, sha: str):
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def load_traffic_sort_join(workload: str):
    """HBM bytes per launch of the sort join's join kernel from the committed
    counter summary, or None when absent or taken on other kernel sources."""
    return _counter_summary(os.path.join(ROOT, "profiles", f"sort_join_{workload}_hbm_counters.md"),
                            kernel_source_hash_sort_join())


def probe_summary_path(workload: str, binned: bool, index: str = "rmi",
                       root: str = "linear") -> str:
    """Committed rocprofv3 counter summary of one probe form."""
    kind = (("probe_binned" if binned else "probe") + ("" if index == "rmi" else "_" + index)
            + ("" if root == "linear" else "_" + root))
    return os.path.join(ROOT, "profiles", f"{kind}_{workload}_hbm_counters.md")


def _summary_value(path: str, key: str):
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def load_traffic(workload: str, binned: bool, index: str = "rmi", root: str = "linear"):
    """HBM bytes per launch of the timed kernel from the committed rocprofv3
    counter summary, or None when absent or taken on a different kernel
    source."""
    return _summary_value(probe_summary_path(workload, binned, index, root),
                          "traffic_bytes_per_launch")


def load_step_traffic(workload: str, binned: bool, index: str = "rmi", root: str = "linear"):
    """HBM bytes of a whole probe step (every library kernel) from the same
    counter summary, or None."""
    return _summary_value(probe_summary_path(workload, binned, index, root), "step_bytes")


def make_workload(name: str):
    import workloads
    if name == "lognormal-zipf-200M":
        return workloads.c2_lognormal_zipf()
    if name == "uniform-1M":
        return workloads.c1_uniform()
    if name == "dup-runs-100M":
        return workloads.c3_dup_runs()
    if name == "seq-holes-200M":
        return workloads.c6_seq_holes()
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(pairs_dev, count: int, m: int, out_per_key: float = 0.0,
                      out_per_pair: float = 8.0, slot_bytes: int = 8) -> float:
    """Compulsory HBM bytes of one launch of the probe kernel: 8 B per outer
    key read, one 64 B sector of the searched array per outer key (its
    insertion point, or every sector its match run spans), and its output:
    8 B per emitted pair (fused probe), or out_per_key bytes of per-key
    result (search kernel of the binned probe).  The searched array is R
    (8 B per key), a gapped RMI's slots or a learned hash's buckets (16 B
    per key of R: slot_bytes = 16).  Computed from
    the emitted pairs: a key with matches owns one contiguous run of r
    indices, and of slots."""
    import torch
    sectors = float(m)
    if count:
        p = pairs_dev[:count].to(torch.int64)
        s, r = p[:, 0], p[:, 1]
        new = torch.ones(count, dtype=torch.bool, device=p.device)
        new[1:] = s[1:] != s[:-1]
        last = torch.ones(count, dtype=torch.bool, device=p.device)
        last[:-1] = new[1:]
        per = 64 // slot_bytes
        span = (r[last] // per - r[new] // per + 1).sum().item()
        sectors += float(span) - float(new.sum().item())
    return 8.0 * m + 64.0 * sectors + out_per_key * m + out_per_pair * count


def host_threads() -> int:
    """Host threads for the oracle's all-cores leg: the CPUs this process may
    run on, at most 16 (one GPU's share of a GPU machine's host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_slices(fn, jobs, threads: int):
    """Run fn(job) for every job in `threads` host threads (the oracle's C
    routines release the interpreter lock); returns (results, seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    if threads == 1:
        out = [fn(j) for j in jobs]
    else:
        with ThreadPoolExecutor(threads) as ex:
            out = list(ex.map(fn, jobs))
    return out, time.perf_counter() - t0


def cpu_baseline(R, S, one_thread_sample: int, threads: int | None = None):
    """The oracle's sort-merge join, timed on the host: on all host cores
    (S cut into one contiguous slice per thread, each slice joined with all
    of R by the unchanged single-threaded oracle; P is the concatenation of
    the slices' results with s offsets) over all of S, and on one thread
    over the first `one_thread_sample` keys of S."""
    import oracle
    threads = threads or host_threads()
    m = len(S)
    cuts = np.linspace(0, m, threads + 1).astype(np.int64)
    counts, dt = _oracle_slices(lambda ab: len(oracle.sort_merge_join(R, S[ab[0]:ab[1]])),
                                list(zip(cuts[:-1], cuts[1:])), threads)
    res = {"value": m / dt, "unit": "probes/s", "cores": threads, "kind": "oracle",
           "sample": f"sort-merge join of all {m} outer keys against all {len(R)} inner keys "
                     f"({sum(counts)} pairs) in {dt:.2f} s, S cut into {threads} slices joined "
                     f"in {threads} host threads"}
    k = min(one_thread_sample, m)
    if k:
        t0 = time.perf_counter()
        P = oracle.sort_merge_join(R, S[:k])
        dt1 = time.perf_counter() - t0
        res["one_thread"] = {"value": k / dt1, "unit": "probes/s", "cores": 1,
                             "sample": f"first {k} outer keys against all {len(R)} inner keys "
                                       f"({len(P)} pairs) in {dt1:.2f} s"}
    return res


def measure_bw_rand(stream, gib: int = 4, granule: int = 64, reads: int = 1 << 28) -> dict:
    """Random-access ceiling on this GPU: lj_bench_random_gather reads
    `reads` 8-byte words, each from a pseudo-random `granule`-byte granule of
    a `gib`-GiB buffer; median of 3 timed launches.  BW_rand counts the whole
    granule per read (the 64-byte sector a probe's search must fetch)."""
    import torch
    from paper_2111_08824_amd import lj
    buf = torch.empty(gib << 30, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    lj.lj_bench_random_gather(buf, granule, reads, 1, sink, stream)
    times = []
    for r in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lj.lj_bench_random_gather(buf, granule, reads, 2 + r, sink, stream)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    del buf
    t = float(np.median(times))
    return {"gbs": round(reads * granule / t / 1e9, 1), "loads_per_s": reads / t,
            "buffer_gib": gib, "granule": granule, "reads": reads}


def random_roofline(value: float, b_probe: float, bw: dict) -> dict:
    """Probes/s ceiling of the random-access roofline (BW_rand / B_probe) and
    the fraction of it reached."""
    roof = bw["gbs"] * 1e9 / b_probe
    return {"bw_rand_gbs": bw["gbs"], "b_probe": round(b_probe, 3),
            "random_roofline_probes_per_s": roof, "frac_random": round(value / roof, 4),
            "nominal_roofline_probes_per_s": HBM_PEAK_GBS * 1e9 / b_probe}


def latency_reps(step, reps: int):
    """p50 / p99 of `reps` synchronous steps (milliseconds)."""
    lat = []
    for _ in range(reps):
        a = time.perf_counter()
        step()
        lat.append(time.perf_counter() - a)
    lat_ms = np.array(lat) * 1e3
    return {"p50": round(float(np.percentile(lat_ms, 50)), 4),
            "p99": round(float(np.percentile(lat_ms, 99)), 4), "reps": reps}


def cpu_baseline_sort_join(w, sample: int):
    import oracle
    R, S = w.R[:sample], w.S[:sample]
    t0 = time.perf_counter()
    P = oracle.sort_join(R, S)
    dt = time.perf_counter() - t0
    return {"value": (len(R) + len(S)) / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"sort join (qsort of both sides, merge) of the first {len(R)} keys of "
                      f"the shuffled R with the first {len(S)} keys of S ({len(P)} pairs) in "
                      f"{dt:.2f} s, one thread"}


def bench_sort_join(args) -> None:
    """Learned sort join (Section IV) of the workload with R shuffled: one
    step = one lj_sort_join_async of both whole relations (model, partition,
    sort, join, emission) plus the count readback."""
    import torch
    import workloads
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    w = workloads.shuffled_inner(make_workload(args.workload))
    n, m = len(w.R), len(w.S)
    print(f"[bench] workload {w.name}: n={n} m={m} ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    r_dev, s_dev = lj.to_device_keys(w.R), lj.to_device_keys(w.S)
    ws = torch.empty(lj.lj_sort_join_workspace_bytes(n, m), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    cnt_host = torch.zeros(1, dtype=torch.int64, pin_memory=True)
    cap = w.expected_count if w.expected_count is not None else 0
    if not cap:
        lj.lj_sort_join_async(r_dev, s_dev, None, cnt, ws, stream)
        cap = int(cnt.item())
    out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda")

    def step():
        lj.lj_sort_join_async(r_dev, s_dev, out, cnt, ws, stream)
        cnt_host.copy_(cnt, non_blocking=True)
        stream.synchronize()
        return int(cnt_host.item())

    for _ in range(args.warmup):
        count = step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for a, b in ev:
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        lj.lj_probe_set_timing_events(ev[i][0], ev[i][1])
        count = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    if w.expected_count is not None and count != w.expected_count:
        raise SystemExit(f"pair count {count} != expected {w.expected_count}")
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    latency = latency_reps(step, max(args.latency_reps, args.steps))
    copy_calibration(args)
    # Join kernel: per key of S its key (8 B) and partition number (4 B)
    # read, one 64 B sector of the sorted R searched, an 8 B result written.
    alg = 84.0 * m
    achieved = alg / (kern_ms * 1e-3) / 1e9
    traffic = load_traffic_sort_join(w.name)
    # A join of two unsorted relations reads each once and writes its pairs:
    # 8 (n + m) + 8 pairs bytes at the least.
    step_alg = 8.0 * (n + m) + 8.0 * count
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg, "kernel": "sj_join_kernel",
            "kernel_ms": round(kern_ms, 4),
            "traffic_gbs": round(traffic / (kern_ms * 1e-3) / 1e9, 1) if traffic else None,
            "step_algorithmic_bytes": step_alg,
            "frac_step": round(step_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del ws, out
    torch.cuda.synchronize()
    cpu = (cpu_baseline_sort_join(w, min(args.cpu_sample, n, m)) if args.cpu_sample
           else None)
    res = {
        "metric": "join tuples/sec ((|R| + |S|) per second), learned sort join",
        "value": (n + m) / (ms_per_step * 1e-3),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "m": m, "join": "learned-sort",
                   "pairs": int(count)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_ms": latency,
    }
    print(json.dumps(res), flush=True)


def root_flag(args) -> int:
    from paper_2111_08824_amd import lj
    return lj.LJ_ROOT_RADIX if args.root == "radix" else 0


def copy_calibration(args) -> None:
    """Three plain device copies of --copy-calibration-mib MiB after the
    timed work: the reference that scales HBM byte counters."""
    if not args.copy_calibration_mib:
        return
    import torch
    src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _json_line(res: dict) -> None:
    print(json.dumps(res), flush=True)


def bench_multi_index(args) -> None:
    """64 independent indexes, one batch of outer keys each, three ways: the
    plain probe launched batch after batch synchronously (lj_probe_join: a
    count readback and a stream wait per batch, as a caller without the
    batched API), the same launches back to back asynchronously on one
    stream (lj_probe_join_async, one wait at the end: device work only), and
    one autotuned plan replayed from a HIP graph (the timed value)."""
    import torch
    import workloads
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    ws = workloads.multi_index_batches(k=64)
    print(f"[bench] generated 64 indexes, {sum(len(w.R) for w in ws)} inner and "
          f"{sum(len(w.S) for w in ws)} outer keys ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    batches, expected, wspaces = [], [], []
    for w in ws:
        ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32 | root_flag(args), stream)
        s = lj.to_device_keys(w.S)
        out = torch.empty((max(1, len(w.S)), 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        batches.append((ix, s, out, cnt))
        expected.append(w.expected_count)
        wspaces.append(torch.empty(max(256, lj.lj_probe_workspace_bytes(ix, len(w.S))),
                                   dtype=torch.uint8, device="cuda"))
    m_total = sum(len(w.S) for w in ws)
    torch.cuda.synchronize()

    def plain_sync():
        for ix, s, out, cnt in batches:
            st, c = lj.lj_probe_join(ix, s, out, stream)
            assert st == lj.LJ_OK

    def plain_async():
        for (ix, s, out, cnt), wsp in zip(batches, wspaces):
            lj.lj_probe_join_async(ix, s, out, cnt, wsp, stream)
        stream.synchronize()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3 / args.steps

    sync_ms = timed(plain_sync)
    async_ms = timed(plain_async)

    tuning = lj.lj_batch_autotune(batches, stream)
    plan = lj.BatchPlan(batches, tuning)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def plan_step():
        plan.run(stream)
        stream.synchronize()

    for _ in range(args.warmup):
        plan_step()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        plan.run(stream)
        ev[i][1].record(stream)
        stream.synchronize()
    plan_ms = (time.perf_counter() - a) * 1e3 / args.steps
    dev_ms = float(np.mean([x.elapsed_time(y) for x, y in ev]))
    got = [int(c.item()) for *_, c in batches]
    if got != expected:
        raise SystemExit("batched pair counts differ from the generator's hit counts")
    latency = latency_reps(plan_step, max(args.latency_reps, args.steps))
    copy_calibration(args)
    value = m_total / (plan_ms * 1e-3)
    alg = sum(algorithmic_bytes(out, c, s.numel()) for (_, s, out, _), c in zip(batches, got))
    achieved = alg / (dev_ms * 1e-3) / 1e9
    # HBM bytes of one replay from the committed counter summary, when it
    # was taken on the current kernel sources and the plan is one fused
    # launch (every index here is a plain FP32 RMI without duplicates, so
    # a fused plan with no binned batch is one launch; the summary counts
    # that launch's kernels).
    one_launch = tuning.fused == 1 and tuning.binned_min_keys in (0, 2**64 - 1)
    traffic = (_summary_value(os.path.join(ROOT, "profiles",
                                           "batched_fused_multi-index-64_hbm_counters.md"),
                              "traffic_bytes_per_launch")
               if args.root == "radix" and one_launch else None)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": alg,
            "kernel": "plan run (graph replay of every batch's probe kernels)",
            "kernel_ms": round(dev_ms, 4),
            "traffic_gbs": round(traffic / (dev_ms * 1e-3) / 1e9, 1) if traffic else None,
            "frac_step": round(alg / (plan_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if args.diagnostics:
        roof.update(random_roofline(value, alg / m_total, measure_bw_rand(stream)))
    plan.close()
    del wspaces
    torch.cuda.synchronize()
    cpu = None
    if args.cpu_sample:
        import oracle
        th = host_threads()
        order = sorted(range(len(ws)), key=lambda i: -len(ws[i].S))  # longest first
        counts, dt = _oracle_slices(lambda i: len(oracle.sort_merge_join(ws[i].R, ws[i].S)),
                                    order, th)
        cpu = {"value": m_total / dt, "unit": "probes/s", "cores": th, "kind": "oracle",
               "sample": f"sort-merge join of all 64 batches ({m_total} outer keys, "
                         f"{sum(counts)} pairs) in {dt:.2f} s, one batch per host thread at "
                         f"a time, {th} threads"}
    _json_line({
        "metric": METRIC, "value": value, "unit": "probes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(plan_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "multi-index-64", "indexes": 64,
                   "inner_keys": int(sum(len(w.R) for w in ws)), "outer_keys": int(m_total),
                   "leaf_model": "fp32", "root": args.root, "tuning": tuning.as_dict()},
        "plain_per_batch_sync": {"ms_per_step": round(sync_ms, 4),
                                 "probes_per_s": m_total / (sync_ms * 1e-3)},
        "plain_per_batch_async": {"ms_per_step": round(async_ms, 4),
                                  "probes_per_s": m_total / (async_ms * 1e-3)},
        "speedup_vs_plain_sync": round(sync_ms / plan_ms, 3),
        "speedup_vs_plain_async": round(async_ms / plan_ms, 3),
        "latency_ms": latency,
        "roofline": roof, "cpu_baseline": cpu,
    })


def bench_serving(args) -> None:
    """8 resident indexes of 5e7 keys, a Poisson stream of requests of
    256..4M keys (log-uniform) at 0.5x and 0.8x the saturation rate of the
    plain per-request probe, run through the serving loop configured as the
    plain per-request probe (one stream, one request per launch) and as the
    continuously batching server (8 streams, up to 16 requests and 2^22 keys
    per batch), with and without the binned probe for requests of 2^20 keys
    or more.  The value is the best served configuration's throughput at
    saturation (all requests submitted at once).  --request-buffers host
    puts request keys and pairs in pinned host memory (PCIe copies
    included) instead of device memory."""
    import threading
    import queue as pyqueue

    import torch
    import workloads
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    ws = workloads.resident_indexes()
    flags = lj.LJ_LEAF_FP32 | root_flag(args)
    if args.index == "gapped":
        ixs = [lj.lj_build_gapped_rmi(w.R, w.leaves, args.slots_per_key, flags) for w in ws]
    elif args.index == "hash":
        ixs = [lj.lj_build_learned_hash(w.R, w.leaves, args.slots_per_key, flags) for w in ws]
    else:
        ixs = [lj.lj_build_rmi(w.R, w.leaves, flags) for w in ws]
    print(f"[bench] 8 resident indexes ready ({args.index}, "
          f"{time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    rng = np.random.default_rng(7)
    max_m = 4 << 20
    nreq = args.requests

    def make_requests(n):
        out = []
        for _ in range(n):
            i = int(rng.integers(0, len(ws)))
            m = int(np.exp(rng.uniform(np.log(256), np.log(max_m))))
            a = int(rng.integers(0, len(ws[i].S) - m))
            out.append((i, a, m))
        return out

    # Outer-key pools in pinned host memory (requests are views into them) and
    # a ring of pinned output buffers; or both in device memory.
    on_device = args.request_buffers == "device"
    pool = len(ws[0].S)
    nbuf = 32
    if on_device:
        s_dev = torch.empty((len(ws), pool), dtype=torch.int64, device="cuda")
        for i, w in enumerate(ws):
            s_dev[i] = lj.to_device_keys(w.S)
        o_dev = torch.empty((nbuf, max_m, 2), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
    else:
        pin_s = torch.empty((len(ws), pool), dtype=torch.int64, pin_memory=True)
        s_np = pin_s.numpy().view(np.uint64)
        for i, w in enumerate(ws):
            s_np[i] = w.S
        pin_o = torch.empty((nbuf, max_m, 2), dtype=torch.int32, pin_memory=True)
        o_np = pin_o.numpy().view(np.uint32)

    if on_device:
        o_all = torch.empty((nreq * (max_m // 8) + max_m, 2), dtype=torch.int32, device="cuda")

    def run_native(cfg, reqs, rate):
        """Device requests submitted by the library's own load driver
        (lj_server_replay: a native thread submits at the arrival times,
        another waits), so that the client costs nothing per request."""
        srv = lj.Server(ixs, cfg)
        items, off = [], 0
        for i, a, m in reqs:
            if off + m > o_all.shape[0]:
                off = 0  # reuse: pairs of early requests are not read back
            items.append((i, s_dev[i, a:a + m], o_all[off:off + m]))
            off += m
        arrival = None
        if rate:
            arrival = np.cumsum(rng.exponential(1.0 / rate, len(reqs))) * 1e9
        torch.cuda.synchronize()
        start = time.perf_counter()
        res = srv.replay(items, arrival)
        wall = time.perf_counter() - start
        assert all(r.status == lj.LJ_OK for r in res)
        lat = np.array([(r.done_ns - r.submit_ns) * 1e-6 for r in res])
        pairs = sum(int(r.count) for r in res)
        st = srv.stats
        srv.close()
        return wall, lat, st, pairs

    def run(cfg, reqs, rate):
        """Submit reqs (Poisson arrivals at `rate` per second, or all at once
        when rate is None); returns (wall seconds, latencies in ms, stats,
        total pairs)."""
        if on_device and args.driver == "native":
            return run_native(cfg, reqs, rate)
        srv = lj.Server(ixs, cfg)
        free = pyqueue.Queue()
        for b in range(nbuf):
            free.put(b)
        tickets = pyqueue.Queue()
        lat = []
        pairs = [0]

        def collector():
            for _ in range(len(reqs)):
                t, b, m = tickets.get()
                r = srv.wait(t)
                assert r.status == lj.LJ_OK
                lat.append((r.done_ns - r.submit_ns) * 1e-6)
                pairs[0] += r.count
                free.put(b)

        th = threading.Thread(target=collector)
        th.start()
        start = time.perf_counter()
        next_t = start
        for i, a, m in reqs:
            if rate:
                next_t += rng.exponential(1.0 / rate)
                d = next_t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
            b = free.get()
            if on_device:
                t = srv.submit_device(i, s_dev[i, a:a + m], o_dev[b, :m])
            else:
                t = srv.submit(i, s_np[i, a:a + m], o_np[b, :m])
            tickets.put((t, b, m))
        th.join()
        wall = time.perf_counter() - start
        st = srv.stats
        srv.close()
        return wall, np.array(lat), st, pairs[0]

    plain = lj.lj_server_default_config(24 << 30)
    plain.slots, plain.max_batch_requests = 1, 1
    served = lj.lj_server_default_config(24 << 30)
    served_binned = lj.lj_server_default_config(24 << 30)
    served_binned.binned_min_keys = 1 << 20
    for c in (served, served_binned):
        if args.serve_slots:
            c.slots = args.serve_slots
        if args.serve_batch_requests:
            c.max_batch_requests = args.serve_batch_requests
        if args.serve_batch_keys:
            c.max_batch_keys = args.serve_batch_keys
    if args.serve_kpl:
        for c in (plain, served, served_binned):
            c.keys_per_lane[:] = [int(v) for v in args.serve_kpl.split(",")]
    configs = [("plain_per_request", plain), ("served", served),
               ("served_binned", served_binned)]

    warm = make_requests(64)
    for _, cfg in configs:
        run(cfg, warm, None)
    sat_reqs = make_requests(nreq)
    keys_sat = sum(m for _, _, m in sat_reqs)
    sat = {}
    for name, cfg in configs:
        wall, lat, st, pairs = run(cfg, sat_reqs, None)
        sat[name] = (wall, st, pairs, lat)
        print(f"[bench] saturation {name}: {len(sat_reqs) / wall:.1f} req/s, "
              f"{keys_sat / wall:.3e} probes/s", file=sys.stderr, flush=True)
    w_plain = sat["plain_per_request"][0]
    best = min((n for n, _ in configs if n != "plain_per_request"), key=lambda n: sat[n][0])
    w_served, st_sat, pairs_sat, lat_sat = sat[best]
    sat_rate = len(sat_reqs) / w_plain
    loads = {}
    for load in (0.5, 0.8):
        reqs = make_requests(nreq)
        keys = sum(m for _, _, m in reqs)
        row = {}
        for name, cfg in configs:
            wall, lat, st, _ = run(cfg, reqs, load * sat_rate)
            row[name] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "probes_per_s": keys / wall, "batches": int(st.batches),
                         "max_batch": int(st.max_batch_size)}
            print(f"[bench] load {load} {name}: {row[name]}", file=sys.stderr, flush=True)
        loads[str(load)] = row
    value = keys_sat / w_served
    # Every resident R is duplicate-free: one sector of R per outer key, at
    # most one pair.
    alg = 72.0 * keys_sat + 8.0 * pairs_sat
    achieved = alg / w_served / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "algorithmic_bytes_per_launch": alg,
            "kernel": f"every probe kernel of the {best} configuration at saturation "
                      "(wall clock)",
            "kernel_ms": round(w_served * 1e3, 3),
            "frac_step": round(achieved / HBM_PEAK_GBS, 4)}
    if args.diagnostics:
        roof.update(random_roofline(value, alg / keys_sat, measure_bw_rand(
            torch.cuda.current_stream())))
        roof["plain_per_request_frac_random"] = round(
            keys_sat / w_plain / roof["random_roofline_probes_per_s"], 4)
    cpu = None
    if args.cpu_sample:
        import oracle
        th = host_threads()
        sample = sat_reqs[:100]
        counts, dt = _oracle_slices(
            lambda r: len(oracle.sort_merge_join(ws[r[0]].R, ws[r[0]].S[r[1]:r[1] + r[2]])),
            sample, th)
        keys = sum(m for _, _, m in sample)
        cpu = {"value": keys / dt, "unit": "probes/s", "cores": th, "kind": "oracle",
               "sample": f"sort-merge join of the first 100 saturation requests ({keys} "
                         f"outer keys, {sum(counts)} pairs) in {dt:.2f} s, one request per "
                         f"host thread at a time, {th} threads"}
    _json_line({
        "metric": METRIC, "value": value, "unit": "probes/s",
        "n_gpus": 1, "steps": len(sat_reqs), "warmup": 0,
        "ms_per_step": round(w_served * 1e3 / len(sat_reqs), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving-8x50M", "indexes": 8, "inner_keys_each": 50_000_000,
                   "index": args.index, "leaf_model": "fp32", "root": args.root,
                   "request_keys": "log-uniform 256..4194304", "requests_per_load": nreq,
                   "request_buffers": args.request_buffers, "server": best,
                   "slots": int(served.slots), "max_batch_requests": int(served.max_batch_requests),
                   "max_batch_keys": int(served.max_batch_keys),
                   "keys_per_lane": [int(v) for v in served.keys_per_lane],
                   "driver": args.driver if on_device else "python"},
        "saturation": {**{f"{n}_probes_per_s": keys_sat / sat[n][0] for n, _ in configs},
                       "served_max_batch": int(st_sat.max_batch_size),
                       "served_speedup_vs_plain": round(w_plain / w_served, 3)},
        "latency_ms": {"p50": round(float(np.percentile(lat_sat, 50)), 4),
                       "p99": round(float(np.percentile(lat_sat, 99)), 4),
                       "reps": len(sat_reqs), "at": "saturation"},
        "loads": loads,
        "roofline": roof, "cpu_baseline": cpu,
    })


def search_diagnostics(ix, R, S, sample: int = 1_000_000, seed: int = 5) -> dict:
    """Model-quality cost of the last-mile search, exactly on the host for a
    sample of the outer keys: the window the index gives each key
    (lj_predict_windows_host, the host copy of the model), then a textbook
    lower_bound over that window of R, counting its probes and the distinct
    64-byte sectors of R they touch (sigma-bar: the paper's last-mile search
    steps, turned into memory sectors)."""
    from paper_2111_08824_amd import lj
    rng = np.random.default_rng(seed)
    k = min(sample, len(S))
    xs = S[rng.choice(len(S), k, replace=False)] if k < len(S) else S
    _, _, lo, hi = lj.lj_predict_windows_host(ix, xs)
    first = np.where(lo <= hi, lo, 0).astype(np.int64)
    win = np.where(lo <= hi, hi - lo + 1, 0).astype(np.int64)
    length = win.copy()
    sect = []
    steps = np.zeros(k, dtype=np.int64)
    while True:
        act = length > 0
        if not act.any():
            break
        half = length >> 1
        mid = np.where(act, first + half, 0)
        sect.append(np.where(act, mid // 8, -1))
        steps += act
        lt = act & (R[mid] < xs)
        first = np.where(lt, mid + 1, first)
        length = np.where(act, np.where(lt, length - half - 1, half), 0)
    if sect:
        a = np.sort(np.stack(sect), axis=0)
        distinct = ((a[1:] != a[:-1]) & (a[1:] >= 0)).sum(axis=0) + (a[0] >= 0)
    else:
        distinct = np.zeros(k, dtype=np.int64)
    return {"sample_keys": int(k), "mean_search_steps": round(float(steps.mean()), 3),
            "sigma_bar_sectors": round(float(distinct.mean()), 3),
            "mean_window_of_sample": round(float(win.mean()), 2)}


def infinite_cache_floor(R, s_dev, out, count: int, m: int) -> dict | None:
    """Compulsory bytes with unlimited cache reuse: 8 B per outer key, one
    64-byte sector of R per distinct sector that any key's insertion point or
    match run falls in (Zipf reuse makes many keys share one), 8 B per pair.
    Positions come from a sorted search of all outer keys in R on the device
    (a diagnostic outside the probe; it needs every key below 2^63, where
    int64 order is uint64 order)."""
    import torch
    from paper_2111_08824_amd import lj
    if (len(R) and int(R[-1]) >= 2**63) or m == 0:
        return None
    r_dev = lj.to_device_keys(R)
    if int(s_dev.min().item()) < 0:
        return None
    pos = torch.searchsorted(r_dev, s_dev)
    sec = torch.clamp(pos, max=max(len(R) - 1, 0)) // 8
    if count:
        sec = torch.cat([sec, out[:count, 1].to(torch.int64) // 8])
    distinct = int(torch.unique(sec).numel())
    del r_dev, pos, sec
    floor = 8.0 * m + 64.0 * distinct + 8.0 * count
    return {"distinct_sectors": distinct, "floor_bytes": floor, "floor_b_probe": floor / m}


def bench_inlj(args) -> None:
    import torch
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    w = make_workload(args.workload)
    print(f"[bench] workload {w.name}: n={len(w.R)} m={len(w.S)} leaves={w.leaves} "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    flags = (lj.LJ_LEAF_FP32 if args.leaf == "fp32" else lj.LJ_LEAF_FP64) | root_flag(args)
    if args.search == "exponential":
        flags |= lj.LJ_SEARCH_EXPONENTIAL
    binned = args.probe == "binned"
    if binned:
        flags |= lj.LJ_PROBE_BINNED
    stream = torch.cuda.current_stream()
    gapped = args.index == "gapped"
    hashed = args.index == "hash"
    t0 = time.perf_counter()
    if gapped:
        ix = lj.lj_build_gapped_rmi(w.R, w.leaves, args.slots_per_key, flags, stream)
    elif hashed:
        ix = lj.lj_build_learned_hash(w.R, w.leaves, args.slots_per_key, flags, stream)
    else:
        ix = lj.lj_build_rmi(w.R, w.leaves, flags, stream)
    build_s = time.perf_counter() - t0
    st = ix.stats
    s_dev = lj.to_device_keys(w.S)
    m = len(w.S)
    cap = m * int(st.max_mult)
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    print(f"[bench] index built in {build_s:.1f} s: mean window {st.mean_window:.1f}, max "
          f"window {st.max_window}, nonempty leaves {st.nonempty_leaves}, device bytes "
          f"{st.device_bytes}", file=sys.stderr, flush=True)

    def step():
        status, count = lj.lj_probe_join(ix, s_dev, out, stream)
        assert status == lj.LJ_OK
        return count

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for a, b in ev:  # materialise the HIP events; the library re-records them
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        lj.lj_probe_set_timing_events(ev[i][0], ev[i][1])
        count = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    if w.expected_count is not None and count != w.expected_count:
        raise SystemExit(f"pair count {count} != expected {w.expected_count}")
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    value = m / (ms_per_step * 1e-3)
    print(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms per step, timed kernel "
          f"{kern_ms:.3f} ms", file=sys.stderr, flush=True)
    latency = latency_reps(step, max(args.latency_reps, args.steps))
    copy_calibration(args)

    slot_bytes = 16 if gapped or hashed else 8
    # The method's compulsory bytes per step (8 B per outer key, the R
    # sectors of its insertion point or match run, 8 B per pair), and those
    # of the timed kernel: for the binned probe its search (a 4- or 8-byte
    # result per key, no pairs).
    step_alg = algorithmic_bytes(out, int(count), m, slot_bytes=slot_bytes)
    if binned:
        alg = algorithmic_bytes(out, int(count), m, 4.0 if st.max_mult <= 1 else 8.0, 0.0,
                                slot_bytes)
    else:
        alg = step_alg
    achieved = alg / (kern_ms * 1e-3) / 1e9
    # The counter summaries were taken with FP32 leaves, binary search and
    # the default slots per key.
    summary_ok = (args.leaf == "fp32" and args.search == "binary"
                  and (args.index == "rmi" or args.slots_per_key == 4))
    traffic = load_traffic(w.name, binned, args.index, args.root) if summary_ok else None
    step_traffic = (load_step_traffic(w.name, binned, args.index, args.root) if summary_ok
                    else None)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg,
            "kernel": (("probe_binned_gapped_kernel+gapped_queue_kernel"
                        if gapped and st.max_mult <= 1 else "probe_binned_kernel")
                       if binned else
                       ("probe_join_full_kernel" if gapped or hashed or st.max_mult > 1
                        else "probe_join_kernel")),
            "kernel_ms": round(kern_ms, 4),
            "traffic_gbs": round(traffic / (kern_ms * 1e-3) / 1e9, 1) if traffic else None,
            "step_algorithmic_bytes": step_alg,
            "frac_step": round(step_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "step_traffic": step_traffic}
    diag = {}
    if args.diagnostics:
        bw = measure_bw_rand(stream)
        roof.update(random_roofline(value, step_alg / m, bw))
        roof["bw_rand_loads_per_s"] = bw["loads_per_s"]
        if not gapped and not hashed:
            # Pred / Srch split (the paper's runtime breakdown): a kernel that
            # only routes, reads the leaf record and computes the window of
            # every outer key (one 8-byte store per key), in S order.
            wlo = torch.empty(m, dtype=torch.int64, device="cuda")
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            lj.lj_predict_windows(ix, s_dev, None, None, wlo, None, stream)
            a.record(stream)
            lj.lj_predict_windows(ix, s_dev, None, None, wlo, None, stream)
            b.record(stream)
            b.synchronize()
            diag["predict_only_ms"] = round(a.elapsed_time(b), 4)
            del wlo
            diag.update(search_diagnostics(ix, w.R, w.S))
        fl = infinite_cache_floor(w.R, s_dev, out, int(count), m)
        if fl:
            diag.update(fl)
            roof["frac_step_floor"] = round(fl["floor_bytes"] / (ms_per_step * 1e-3) / 1e9
                                            / HBM_PEAK_GBS, 4)
    del out
    torch.cuda.synchronize()

    cpu = (cpu_baseline(w.R, w.S, min(args.cpu_sample, m)) if args.cpu_sample else None)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "probes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": len(w.R), "m": m, "leaves": w.leaves,
                   "leaf_model": args.leaf, "root": args.root,
                   "search": ("gapped-exponential" if gapped else "bucket-chain" if hashed
                              else args.search),
                   "probe": args.probe,
                   "index": args.index,
                   "slots_per_key": args.slots_per_key if gapped or hashed else None,
                   "pairs": int(count),
                   "mean_window": round(st.mean_window, 2), "max_window": int(st.max_window)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_ms": latency,
        "join_tuples_per_s": (len(w.R) + m) / (ms_per_step * 1e-3),
        "diagnostics": diag or None,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal-zipf-200M")
    ap.add_argument("--leaf", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--root", choices=["linear", "radix"], default="radix",
                    help="root model: one least-squares line, or a piecewise-linear CDF "
                         "over a radix table of the key")
    ap.add_argument("--search", choices=["binary", "exponential"], default="binary",
                    help="last-mile search inside the error bounds")
    ap.add_argument("--probe", choices=["direct", "binned"], default="binned",
                    help="probe S in its own order, or partitioned by key range first")
    ap.add_argument("--index", choices=["rmi", "gapped", "hash"], default="rmi",
                    help="plain RMI over R, gapped RMI (model-based insertion), or "
                         "learned hash (the RMI as hash function of a bucket-chained table)")
    ap.add_argument("--slots-per-key", type=int, default=4,
                    help="gapped RMI or learned hash: slots per key of R")
    ap.add_argument("--join", choices=["inlj", "lsj"], default="inlj",
                    help="learned indexed nested loop join (index on sorted R), or the "
                         "learned sort join of R shuffled and S")
    ap.add_argument("--cpu-sample", type=int, default=30_000_000,
                    help="outer keys in the one-thread oracle sample (0 = skip both "
                         "oracle legs); the all-cores leg joins the whole workload")
    ap.add_argument("--latency-reps", type=int, default=100,
                    help="synchronous steps behind p50 / p99 (at least --steps)")
    ap.add_argument("--no-diagnostics", dest="diagnostics", action="store_false",
                    help="skip BW_rand, the predict-only timing, sigma-bar and the "
                         "infinite-cache floor")
    ap.add_argument("--requests", type=int, default=1000,
                    help="requests per load level in the serving workload")
    ap.add_argument("--request-buffers", choices=["host", "device"], default="device",
                    help="serving workload: request keys and pairs already in device "
                         "memory, or in pinned host memory (copied over PCIe)")
    ap.add_argument("--serve-slots", type=int, default=0,
                    help="serving workload: batches in flight (0 = the library default)")
    ap.add_argument("--serve-batch-requests", type=int, default=0,
                    help="serving workload: requests per batch (0 = the library default)")
    ap.add_argument("--serve-batch-keys", type=int, default=0,
                    help="serving workload: outer keys per batch (0 = the library default)")
    ap.add_argument("--serve-kpl", default="",
                    help="serving workload: keys per lane of the four request size classes, "
                         "e.g. 4,8,8,8 (empty = the library default)")
    ap.add_argument("--driver", choices=["native", "python"], default="native",
                    help="serving workload with device buffers: requests submitted by the "
                         "library's native load driver, or one by one from Python threads")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the steps, run a plain device copy of this many MiB "
                         "(reference point for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the probe runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.workload == "multi-index-64":
        return bench_multi_index(args)
    if args.workload == "serving-8x50M":
        return bench_serving(args)
    if args.join == "lsj":
        return bench_sort_join(args)
    return bench_inlj(args)


if __name__ == "__main__":
    main()
