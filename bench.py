#!/usr/bin/env python3
"""Benchmark of the learned indexed nested loop join probe on one MI355X.

One step = one synchronous probe (lj_probe_join) of the whole outer relation
S against the two-level linear RMI over R: root model, leaf model, bounded
last-mile search, match counting, output compaction and pair emission, plus
the 8-byte count readback.  R, the index and S are resident in HBM before
the timed region; building the index is offline (untimed).

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
                        "paper_2111_08824_amd/csrc/rmi_eval.h",
                        "paper_2111_08824_amd/csrc/lj_internal.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in PROBE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per probe launch from the committed rocprofv3 counter summary,
    or None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"probe_{workload}_hbm_counters.md")
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
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(pairs_dev, count: int, m: int) -> float:
    """Compulsory HBM bytes of one probe launch: 8 B per outer key read, one
    64 B sector of R per outer key (its insertion point, or every sector its
    match run spans), and 8 B per emitted pair.  Computed from the emitted
    pairs: a key with matches owns one contiguous run of r indices."""
    import torch
    sectors = float(m)
    if count:
        p = pairs_dev[:count].to(torch.int64)
        s, r = p[:, 0], p[:, 1]
        new = torch.ones(count, dtype=torch.bool, device=p.device)
        new[1:] = s[1:] != s[:-1]
        last = torch.ones(count, dtype=torch.bool, device=p.device)
        last[:-1] = new[1:]
        span = (r[last] // 8 - r[new] // 8 + 1).sum().item()
        sectors += float(span) - float(new.sum().item())
    return 8.0 * m + 64.0 * sectors + 8.0 * count


def cpu_baseline(w, sample: int):
    import oracle
    S = w.S[:sample]
    t0 = time.perf_counter()
    P = oracle.sort_merge_join(w.R, S)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "probes/s", "cores": 1, "kind": "oracle",
            "sample": f"sort-merge join of the first {sample} outer keys against all "
                      f"{len(w.R)} inner keys ({len(P)} pairs) in {dt:.2f} s, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal-zipf-200M")
    ap.add_argument("--leaf", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-sample", type=int, default=120_000_000,
                    help="outer keys in the timed oracle sample (0 = skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the steps, run a plain device copy of this many MiB "
                         "(reference point for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2111_08824_amd import lj

    t0 = time.perf_counter()
    w = make_workload(args.workload)
    print(f"[bench] workload {w.name}: n={len(w.R)} m={len(w.S)} leaves={w.leaves} "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    flags = lj.LJ_LEAF_FP32 if args.leaf == "fp32" else lj.LJ_LEAF_FP64
    stream = torch.cuda.current_stream()
    ix = lj.lj_build_rmi(w.R, w.leaves, flags, stream)
    st = ix.stats
    s_dev = lj.to_device_keys(w.S)
    m = len(w.S)
    cap = m * int(st.max_mult)
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    print(f"[bench] index built: mean window {st.mean_window:.1f}, max window "
          f"{st.max_window}, nonempty leaves {st.nonempty_leaves}", file=sys.stderr, flush=True)

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

    alg = algorithmic_bytes(out, int(count), m)
    achieved = alg / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": load_traffic(w.name),
            "algorithmic_bytes_per_launch": alg,
            "kernel": "probe_join_kernel", "kernel_ms": round(kern_ms, 4)}

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
                   "leaf_model": args.leaf, "pairs": int(count),
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
