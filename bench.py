#!/usr/bin/env python3
"""Benchmark of the learned indexed nested loop join probe on one MI355X.

One step = one synchronous probe (lj_probe_join) of the whole outer relation
S against the two-level linear RMI over R: root model, leaf model, bounded
last-mile search, match counting, output compaction and pair emission, plus
the 8-byte count readback.  R, the index and S are resident in HBM before
the timed region; building the index is offline (untimed).  By default the
probe is the binned one (S partitioned by key range of R first, the same
pairs in the same order); --probe direct probes S in its own order.

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


def load_traffic(workload: str, binned: bool, index: str = "rmi"):
    """HBM bytes per launch of the timed kernel from the committed rocprofv3
    counter summary, or None when absent or taken on a different kernel
    source."""
    kind = ("probe_binned" if binned else "probe") + ("" if index == "rmi" else "_" + index)
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_hbm_counters.md")
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
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def cpu_baseline(w, sample: int):
    import oracle
    S = w.S[:sample]
    t0 = time.perf_counter()
    P = oracle.sort_merge_join(w.R, S)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "probes/s", "cores": 1, "kind": "oracle",
            "sample": f"sort-merge join of the first {sample} outer keys against all "
                      f"{len(w.R)} inner keys ({len(P)} pairs) in {dt:.2f} s, one thread"}


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
    lat = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        lj.lj_probe_set_timing_events(ev[i][0], ev[i][1])
        a = time.perf_counter()
        count = step()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    if w.expected_count is not None and count != w.expected_count:
        raise SystemExit(f"pair count {count} != expected {w.expected_count}")
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # Join kernel: per key of S its key (8 B) and partition number (4 B)
    # read, one 64 B sector of the sorted R searched, an 8 B result written.
    alg = 84.0 * m
    achieved = alg / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": load_traffic_sort_join(w.name),
            "algorithmic_bytes_per_launch": alg, "kernel": "sj_join_kernel",
            "kernel_ms": round(kern_ms, 4)}
    cpu = (cpu_baseline_sort_join(w, min(args.cpu_sample // 4, n, m)) if args.cpu_sample
           else None)
    lat_ms = np.array(lat) * 1e3
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
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
    }
    print(json.dumps(res), flush=True)


def _json_line(res: dict) -> None:
    print(json.dumps(res), flush=True)


def bench_multi_index(args) -> None:
    """64 independent indexes, one batch of outer keys each: the plain probe
    launched batch after batch (synchronous, as a caller would without the
    batched API) against one autotuned plan replayed from a HIP graph."""
    import torch
    import workloads
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    ws = workloads.multi_index_batches(k=64)
    print(f"[bench] generated 64 indexes, {sum(len(w.R) for w in ws)} inner and "
          f"{sum(len(w.S) for w in ws)} outer keys ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    batches, expected = [], []
    for w in ws:
        ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32, stream)
        s = lj.to_device_keys(w.S)
        out = torch.empty((max(1, len(w.S)), 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        batches.append((ix, s, out, cnt))
        expected.append(w.expected_count)
    m_total = sum(len(w.S) for w in ws)
    torch.cuda.synchronize()

    def plain_once():
        for ix, s, out, cnt in batches:
            st, c = lj.lj_probe_join(ix, s, out, stream)
            assert st == lj.LJ_OK

    for _ in range(args.warmup):
        plain_once()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(args.steps):
        plain_once()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - a) * 1e3 / args.steps

    tuning = lj.lj_batch_autotune(batches, stream)
    plan = lj.BatchPlan(batches, tuning)
    for _ in range(args.warmup):
        plan.run(stream)
    torch.cuda.synchronize()
    lat = []
    a = time.perf_counter()
    for _ in range(args.steps):
        b = time.perf_counter()
        plan.run(stream)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - b)
    plan_ms = (time.perf_counter() - a) * 1e3 / args.steps
    got = [int(c.item()) for *_, c in batches]
    if got != expected:
        raise SystemExit("batched pair counts differ from the generator's hit counts")
    lat_ms = np.array(lat) * 1e3
    _json_line({
        "metric": METRIC, "value": m_total / (plan_ms * 1e-3), "unit": "probes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(plan_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "multi-index-64", "indexes": 64,
                   "inner_keys": int(sum(len(w.R) for w in ws)), "outer_keys": int(m_total),
                   "tuning": tuning.as_dict()},
        "plain_per_batch": {"ms_per_step": round(plain_ms, 4),
                            "probes_per_s": m_total / (plain_ms * 1e-3)},
        "speedup_vs_plain": round(plain_ms / plan_ms, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "roofline": None, "cpu_baseline": None,
    })


def bench_serving(args) -> None:
    """8 resident indexes of 5e7 keys, a Poisson stream of requests of
    256..4M keys (log-uniform) at 0.5x and 0.8x the saturation rate of the
    plain per-request probe, run through the serving loop configured as the
    plain per-request probe (one stream, one request per launch) and as the
    continuously batching server (8 streams, up to 16 requests and 2^22 keys
    per batch).  --request-buffers device keeps request keys and pairs in
    HBM (lj_server_submit_device: no PCIe copies) and adds a server
    configuration that probes requests of 2^20 keys or more binned."""
    import threading
    import queue as pyqueue

    import torch
    import workloads
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    ws = workloads.resident_indexes()
    ixs = [lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32) for w in ws]
    print(f"[bench] 8 resident indexes ready ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
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

    def run(cfg, reqs, rate):
        """Submit reqs (Poisson arrivals at `rate` per second, or all at once
        when rate is None); returns (wall seconds, latencies in ms)."""
        srv = lj.Server(ixs, cfg)
        free = pyqueue.Queue()
        for b in range(nbuf):
            free.put(b)
        tickets = pyqueue.Queue()
        lat = []

        def collector():
            for _ in range(len(reqs)):
                t, b, m = tickets.get()
                r = srv.wait(t)
                assert r.status == lj.LJ_OK
                lat.append((r.done_ns - r.submit_ns) * 1e-6)
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
        return wall, np.array(lat), st

    plain = lj.lj_server_default_config(24 << 30)
    plain.slots, plain.max_batch_requests = 1, 1
    served = lj.lj_server_default_config(24 << 30)
    configs = [("plain_per_request", plain), ("served", served)]
    if on_device:
        served_binned = lj.lj_server_default_config(24 << 30)
        served_binned.binned_min_keys = 1 << 20
        configs.append(("served_binned", served_binned))

    warm = make_requests(64)
    for _, cfg in configs:
        run(cfg, warm, None)
    sat_reqs = make_requests(nreq)
    keys_sat = sum(m for _, _, m in sat_reqs)
    sat = {}
    for name, cfg in configs:
        wall, _, st = run(cfg, sat_reqs, None)
        sat[name] = (wall, st)
        print(f"[bench] saturation {name}: {len(sat_reqs) / wall:.1f} req/s, "
              f"{keys_sat / wall:.3e} probes/s", file=sys.stderr, flush=True)
    w_plain = sat["plain_per_request"][0]
    best = min((n for n, _ in configs if n != "plain_per_request"), key=lambda n: sat[n][0])
    w_served, st_sat = sat[best]
    sat_rate = len(sat_reqs) / w_plain
    loads = {}
    for load in (0.5, 0.8):
        reqs = make_requests(nreq)
        keys = sum(m for _, _, m in reqs)
        row = {}
        for name, cfg in configs:
            wall, lat, st = run(cfg, reqs, load * sat_rate)
            row[name] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "probes_per_s": keys / wall, "batches": int(st.batches),
                         "max_batch": int(st.max_batch_size)}
            print(f"[bench] load {load} {name}: {row[name]}", file=sys.stderr, flush=True)
        loads[str(load)] = row
    _json_line({
        "metric": METRIC, "value": keys_sat / w_served, "unit": "probes/s",
        "n_gpus": 1, "steps": len(sat_reqs), "warmup": 0,
        "ms_per_step": round(w_served * 1e3 / len(sat_reqs), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving-8x50M", "indexes": 8, "inner_keys_each": 50_000_000,
                   "request_keys": "log-uniform 256..4194304", "requests_per_load": nreq,
                   "request_buffers": args.request_buffers, "server": best},
        "saturation": {**{f"{n}_probes_per_s": keys_sat / sat[n][0] for n, _ in configs},
                       "served_max_batch": int(st_sat.max_batch_size)},
        "loads": loads,
        "roofline": None, "cpu_baseline": None,
    })


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal-zipf-200M")
    ap.add_argument("--leaf", choices=["fp32", "fp64"], default="fp32")
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
    ap.add_argument("--cpu-sample", type=int, default=120_000_000,
                    help="outer keys in the timed oracle sample (0 = skip)")
    ap.add_argument("--requests", type=int, default=1000,
                    help="requests per load level in the serving workload")
    ap.add_argument("--request-buffers", choices=["host", "device"], default="host",
                    help="serving workload: request keys and pairs in pinned host memory "
                         "(copied over PCIe) or already in device memory")
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

    import torch
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    w = make_workload(args.workload)
    print(f"[bench] workload {w.name}: n={len(w.R)} m={len(w.S)} leaves={w.leaves} "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    flags = lj.LJ_LEAF_FP32 if args.leaf == "fp32" else lj.LJ_LEAF_FP64
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

    for _ in range(args.warmup):
        status, count = lj.lj_probe_join(ix, s_dev, out, stream)
        assert status == lj.LJ_OK
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for a, b in ev:  # materialise the HIP events; the library re-records them
        a.record(stream)
        b.record(stream)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        lj.lj_probe_set_timing_events(ev[i][0], ev[i][1])
        a = time.perf_counter()
        status, count = lj.lj_probe_join(ix, s_dev, out, stream)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    assert status == lj.LJ_OK
    if w.expected_count is not None and count != w.expected_count:
        raise SystemExit(f"pair count {count} != expected {w.expected_count}")
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps

    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    slot_bytes = 16 if gapped or hashed else 8
    if binned:  # search kernel: keys in, one 4-byte (8 with duplicates) result out
        alg = algorithmic_bytes(out, int(count), m, 4.0 if st.max_mult <= 1 else 8.0, 0.0,
                                slot_bytes)
    else:
        alg = algorithmic_bytes(out, int(count), m, slot_bytes=slot_bytes)
    achieved = alg / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            # The counter summaries were taken with FP32 leaves, binary search
            # and the default slots per key.
            "traffic": (load_traffic(w.name, binned, args.index)
                        if args.leaf == "fp32" and args.search == "binary"
                        and (args.index == "rmi" or args.slots_per_key == 4) else None),
            "algorithmic_bytes_per_launch": alg,
            "kernel": (("probe_binned_gapped_kernel+gapped_queue_kernel"
                        if gapped and st.max_mult <= 1 else "probe_binned_kernel")
                       if binned else "probe_join_kernel"),
            "kernel_ms": round(kern_ms, 4)}

    cpu = cpu_baseline(w, min(args.cpu_sample, m)) if args.cpu_sample else None
    lat_ms = np.array(lat) * 1e3
    res = {
        "metric": METRIC,
        "value": m / (ms_per_step * 1e-3),
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
                   "leaf_model": args.leaf,
                   "search": ("gapped-exponential" if gapped else "bucket-chain" if hashed
                              else args.search),
                   "probe": args.probe,
                   "index": args.index,
                   "slots_per_key": args.slots_per_key if gapped or hashed else None,
                   "pairs": int(count),
                   "mean_window": round(st.mean_window, 2), "max_window": int(st.max_window)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "join_tuples_per_s": (len(w.R) + m) / (ms_per_step * 1e-3),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
