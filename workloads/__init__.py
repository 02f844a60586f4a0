"""Seeded synthetic inputs for the learned indexed nested loop join.

This package is shared by the CPU oracle (``oracle/``) and by the GPU library
and holds none of the join's or the index's arithmetic: it only produces the
inner relation R (sorted uint64 keys) and the outer relation S (uint64 probe
keys) of each workload.

The shapes follow the paper's synthetic datasets (Section VI-A, "Datasets"):
``unif`` (uniform keys), ``lognorm`` (lognormal keys) and ``seq_h``
(sequential IDs with 10% random holes), widened to 64-bit keys, plus the
duplicate-run and Zipf-reuse variants of the workloads measured here.
"""
from .gen import (  # noqa: F401
    lib, stream_key, uniform_unique, lognormal_unique, seq_holes, dup_runs,
    probe_mix, permute, shuffle,
)
from .configs import (  # noqa: F401
    Workload, c1_uniform, c2_lognormal_zipf, c3_dup_runs, c6_seq_holes, multi_index_batches,
    shuffled_inner,
    default_leaves, resident_indexes,
)
