"""The threaded equal_range helper that the full-shape GPU tests take their
expected pairs from agrees with the oracle's sort-merge join."""
import numpy as np

import oracle
import workloads
from exact_pairs import equal_range_threaded, expected_pairs_unique


def test_expected_pairs_equal_sort_merge_join():
    for seed in range(3):
        w = workloads.c2_lognormal_zipf(seed=seed, scale=0.001)
        got = expected_pairs_unique(w.R, w.S, threads=4)
        assert np.array_equal(got, oracle.sort_merge_join(w.R, w.S))
        assert len(got) == w.expected_count


def test_threaded_equal_range_equals_one_thread():
    w = workloads.c1_uniform(scale=0.2)
    f1, c1 = oracle.equal_range(w.R, w.S)
    f4, c4 = equal_range_threaded(w.R, w.S, threads=4)
    assert np.array_equal(f1, f4) and np.array_equal(c1, c4)
