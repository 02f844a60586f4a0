"""Named workloads (R, S, leaf count) at full size or scaled down.

Full sizes:
  c1_uniform         R = 1e6 distinct uniform keys in [0, 2^40), 4096 leaves;
                     S = 1e6 keys, 50% hits (uniform, with replacement),
                     50% misses uniform in [0, 2^40).
  c2_lognormal_zipf  R = 2e8 distinct lognormal(0, 2) keys scaled to 2^63,
                     2^20 leaves; S = 2e8 keys, 90% hits by Zipf(1) rank,
                     10% misses uniform in [0, 2^63).
  c3_dup_runs        R = 1e8 rows of seq_h values each repeated U{1..16}
                     times, 2^19 leaves; S = 1e8 keys, 70% hits uniform over
                     the distinct values, 30% misses (holes and values above
                     the largest key).
  c6_seq_holes       R = 2e8 sequential IDs with 10% random holes (seq_h),
                     2^20 leaves; S = 2e8 keys, 90% hits uniform over R,
                     10% misses (holes and values above the largest key).
  multi_index_batches  many independent inner relations of log-uniform size
                     and mixed shape, each probed by one batch of
                     log-uniform size with 50% hits.

``scale`` < 1 shrinks n, m and the leaf count together (for tests).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import gen


@dataclass
class Workload:
    name: str
    R: np.ndarray
    S: np.ndarray
    leaves: int
    expected_count: int | None = None  # exact pair count when the generator fixes it
    meta: dict = field(default_factory=dict)


def default_leaves(n: int) -> int:
    """2^round(log2(n / 256)), clamped to [1, 2^20]."""
    if n <= 256:
        return 1
    return int(min(2**20, max(1, 2 ** round(math.log2(n / 256.0)))))


def _scaled(v: int, scale: float) -> int:
    return max(1, int(round(v * scale)))


def _scaled_leaves(leaves: int, scale: float) -> int:
    return int(max(1, 2 ** round(math.log2(max(1.0, leaves * scale)))))


def c1_uniform(seed: int = 42, scale: float = 1.0) -> Workload:
    n, m = _scaled(1_000_000, scale), _scaled(1_000_000, scale)
    R = gen.uniform_unique(n, 40, seed)
    S = gen.probe_mix(R, m, 0.5, seed + 1, miss_lo=0, miss_hi=2**40)
    return Workload("uniform-1M" if scale == 1.0 else f"uniform-{n}", R, S,
                    _scaled_leaves(4096, scale), int(round(m * 0.5)),
                    {"n": n, "m": m, "hit_frac": 0.5, "dist": "uniform[0,2^40)"})


def c2_lognormal_zipf(seed: int = 42, scale: float = 1.0) -> Workload:
    n, m = _scaled(200_000_000, scale), _scaled(200_000_000, scale)
    R = gen.lognormal_unique(n, 2.0, seed)
    S = gen.probe_mix(R, m, 0.9, seed + 1, zipf_s=1.0, miss_lo=0, miss_hi=2**63)
    return Workload("lognormal-zipf-200M" if scale == 1.0 else f"lognormal-zipf-{n}",
                    R, S, _scaled_leaves(2**20, scale), int(round(m * 0.9)),
                    {"n": n, "m": m, "hit_frac": 0.9, "dist": "lognormal(0,2)->2^63",
                     "hits": "zipf(1.0)"})


def c3_dup_runs(seed: int = 42, scale: float = 1.0) -> Workload:
    rows, m = _scaled(100_000_000, scale), _scaled(100_000_000, scale)
    R = gen.dup_runs(rows, seed)
    top = int(R[-1])
    S = gen.probe_mix(R, m, 0.7, seed + 1, miss_lo=0, miss_hi=top + top // 8 + 2)
    return Workload("dup-runs-100M" if scale == 1.0 else f"dup-runs-{rows}", R, S,
                    _scaled_leaves(2**19, scale), None,
                    {"n": rows, "m": m, "hit_frac": 0.7, "dist": "seq_h x U{1..16}"})


def c6_seq_holes(seed: int = 42, scale: float = 1.0) -> Workload:
    n, m = _scaled(200_000_000, scale), _scaled(200_000_000, scale)
    R = gen.seq_holes(n, seed)
    top = int(R[-1]) if n else 0
    S = gen.probe_mix(R, m, 0.9, seed + 1, miss_lo=0, miss_hi=top + top // 8 + 2)
    return Workload("seq-holes-200M" if scale == 1.0 else f"seq-holes-{n}", R, S,
                    _scaled_leaves(2**20, scale), int(round(m * 0.9)),
                    {"n": n, "m": m, "hit_frac": 0.9, "dist": "seq_h (10% holes)"})


def shuffled_inner(w: Workload, seed: int = 7) -> Workload:
    """The same workload with R in a seeded random order: the unsorted inner
    relation a sort-based join takes (Section IV).  S is unchanged."""
    R = gen.shuffle(gen.stream_key(seed, 0x5a), w.R)
    return Workload(w.name + "-shuffled", R, w.S, w.leaves, w.expected_count,
                    dict(w.meta, r_order="shuffled"))


def multi_index_batches(k: int = 64, seed: int = 42, n_lo: float = 1e4,
                        n_hi: float = 5e7, m_lo: float = 1e3, m_hi: float = 1e7):
    """k (R, S, leaves) triples: n log-uniform in [n_lo, n_hi], shape chosen
    uniformly among uniform / lognormal / seq_h, m log-uniform in
    [m_lo, m_hi], 50% hits."""
    key = gen.stream_key(seed, 0xC4)
    u = gen.draw_u64(key, 0, 3 * k, 11).astype(np.float64) * 2.0**-53
    out = []
    for i in range(k):
        n = int(math.exp(math.log(n_lo) + u[3 * i] * (math.log(n_hi) - math.log(n_lo))))
        m = int(math.exp(math.log(m_lo) + u[3 * i + 1] * (math.log(m_hi) - math.log(m_lo))))
        shape = int(u[3 * i + 2] * 3)
        s = seed * 1000 + i
        if shape == 0:
            R = gen.uniform_unique(n, 40, s)
            hi = 2**40
        elif shape == 1:
            R = gen.lognormal_unique(n, 2.0, s)
            hi = 2**63
        else:
            R = gen.seq_holes(n, s)
            hi = int(R[-1]) + int(R[-1]) // 8 + 2
        S = gen.probe_mix(R, m, 0.5, s + 1, miss_lo=0, miss_hi=hi)
        out.append(Workload(f"batch{i}-{['uniform', 'lognormal', 'seq_h'][shape]}-{n}",
                            R, S, default_leaves(n), int(round(m * 0.5)),
                            {"n": n, "m": m, "shape": shape}))
    return out


def resident_indexes(k: int = 8, n: int = 50_000_000, pool: int = 8_000_000, seed: int = 42):
    """k inner relations of n keys for the serving workload (3 uniform in
    [0, 2^40), 3 lognormal(0, 2) scaled to 2^63, 2 seq_h, in that rotation),
    each with a pool of outer keys (50% hits) that requests slice."""
    shapes = ["uniform", "uniform", "uniform", "lognormal", "lognormal", "lognormal",
              "seq_h", "seq_h"]
    out = []
    for i in range(k):
        shape = shapes[i % len(shapes)]
        s = seed * 7919 + i
        if shape == "uniform":
            R = gen.uniform_unique(n, 40, s)
            hi = 2**40
        elif shape == "lognormal":
            R = gen.lognormal_unique(n, 2.0, s)
            hi = 2**63
        else:
            R = gen.seq_holes(n, s)
            hi = int(R[-1]) + int(R[-1]) // 8 + 2
        S = gen.probe_mix(R, pool, 0.5, s + 1, miss_lo=0, miss_hi=hi)
        out.append(Workload(f"resident{i}-{shape}-{n}", R, S, default_leaves(n), None,
                            {"n": n, "shape": shape}))
    return out
