"""The benchmark's command line on a host without a GPU: more than one GPU
is refused with a JSON error line, and the algorithmic byte count of a
launch follows its definition on a tiny hand-checked case."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_algorithmic_bytes_definition():
    import torch
    sys.path.insert(0, ROOT)
    import bench
    # 3 outer keys; key 0 matches r 5..9 (one run over sectors 0 and 1 of R:
    # 8 keys per 64-byte sector), key 2 matches r 16; key 1 misses.
    pairs = torch.tensor([[0, 5], [0, 6], [0, 7], [0, 8], [0, 9], [2, 16]], dtype=torch.int32)
    got = bench.algorithmic_bytes(pairs, 6, 3)
    sectors = 3 + (2 - 1) + (1 - 1)  # one per key, plus the extra sector of the run
    assert got == 8 * 3 + 64 * sectors + 8 * 6
    # Binned search kernel: 4 bytes of result per key, no pair bytes.
    assert bench.algorithmic_bytes(pairs, 6, 3, 4.0, 0.0) == 8 * 3 + 64 * sectors + 4 * 3
    # Gapped slots (16 bytes): 4 slots per sector, so r 5..9 spans 2 sectors.
    assert bench.algorithmic_bytes(pairs, 6, 3, slot_bytes=16) == 8 * 3 + 64 * (3 + 1) + 8 * 6


def test_search_diagnostics_count_probes_and_sectors():
    """sigma-bar and the step count of the benchmark's diagnostics equal a
    one-key-at-a-time textbook lower_bound over each key's window, written
    out here with a set of the 64-byte sectors it reads."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads
    from paper_2111_08824_amd import lj
    w = workloads.c2_lognormal_zipf(scale=0.0005)
    ix = lj.lj_build_rmi_host_only(w.R, w.leaves, lj.LJ_LEAF_FP32)
    d = bench.search_diagnostics(ix, w.R, w.S, sample=300, seed=3)
    rng = np.random.default_rng(3)
    xs = w.S[rng.choice(len(w.S), 300, replace=False)]
    _, _, lo, hi = lj.lj_predict_windows_host(ix, xs)
    steps, sectors = [], []
    for x, a, b in zip(xs, lo, hi):
        first, n, seen, k = int(a), int(b - a + 1) if a <= b else 0, set(), 0
        while n > 0:
            half = n // 2
            mid = first + half
            seen.add(mid // 8)
            k += 1
            if w.R[mid] < x:
                first, n = mid + 1, n - half - 1
            else:
                n = half
        steps.append(k)
        sectors.append(len(seen))
    assert d["sample_keys"] == 300
    assert abs(d["mean_search_steps"] - np.mean(steps)) < 1e-3
    assert abs(d["sigma_bar_sectors"] - np.mean(sectors)) < 1e-3
