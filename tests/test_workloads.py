"""Generators: determinism, shapes and exact hit counts (no GPU)."""
import math

import numpy as np
import pytest

import workloads
from workloads import gen


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 1234567 (the published test vector sequence).
    out = gen.draw_u64(1234567, 0, 5)
    assert [int(x) for x in out] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_determinism_and_thread_independence():
    a = workloads.c1_uniform(seed=7, scale=0.05)
    b = workloads.c1_uniform(seed=7, scale=0.05)
    assert np.array_equal(a.R, b.R) and np.array_equal(a.S, b.S)
    c = workloads.c1_uniform(seed=8, scale=0.05)
    assert not np.array_equal(a.S, c.S)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 1000, 4097])
def test_permutation_is_bijection(n):
    p = gen.permute(99, n, np.arange(n, dtype=np.uint64))
    assert np.array_equal(np.sort(p), np.arange(n, dtype=np.uint64))


def test_shuffle_keeps_multiset():
    a = np.arange(1000, dtype=np.uint64) % 37
    s = gen.shuffle(5, a)
    assert np.array_equal(np.sort(s), np.sort(a))
    assert not np.array_equal(s, a)


def test_uniform_unique_shape():
    R = gen.uniform_unique(50_000, 40, 3)
    assert len(R) == 50_000
    assert np.all(R[1:] > R[:-1])
    assert int(R[-1]) < 2**40


def test_lognormal_unique_shape():
    R = gen.lognormal_unique(100_000, 2.0, 3)
    assert len(R) == 100_000 and np.all(R[1:] > R[:-1])
    assert int(R[-1]) <= 2**63 - 1
    # median of lognormal(0, 2) is 1 while the scale maps v_max to 2^63:
    # half of the keys lie far below 2^63 / 1000.
    assert int(R[len(R) // 2]) < 2**63 // 1000


def test_seq_holes_fraction():
    v = gen.seq_holes(100_000, 1)
    assert np.all(v[1:] > v[:-1])
    hole_frac = 1.0 - len(v) / (int(v[-1]) + 1)
    assert abs(hole_frac - 0.1) < 0.01


def test_dup_runs_lengths():
    R = gen.dup_runs(200_000, 2)
    assert len(R) == 200_000 and np.all(R[1:] >= R[:-1])
    _, c = np.unique(R, return_counts=True)
    assert c.min() >= 1 and c[:-1].max() <= 16
    assert abs(c[:-1].mean() - 8.5) < 0.2


@pytest.mark.parametrize("zipf", [None, 1.0])
def test_probe_mix_exact_hits(zipf):
    R = gen.uniform_unique(20_000, 40, 4)
    S = gen.probe_mix(R, 30_001, 0.9, 5, zipf_s=zipf)
    assert len(S) == 30_001
    assert int(np.isin(S, R).sum()) == int(round(30_001 * 0.9))


def test_zipf_rank_frequencies():
    n = 1000
    r = gen.draw_zipf1(77, 400_000, n)
    assert r.min() >= 1 and r.max() <= n
    h = sum(1.0 / k for k in range(1, n + 1))
    for k in (1, 2, 10, 100):
        want = 1.0 / (k * h)
        got = float(np.mean(r == k))
        assert abs(got - want) < 5 * math.sqrt(want / 400_000) + 1e-4, (k, got, want)


def test_workload_defaults():
    assert workloads.default_leaves(1_000_000) == 4096
    assert workloads.default_leaves(200_000_000) == 2**20
    assert workloads.default_leaves(10) == 1


def test_seq_holes_workload_exact_hits():
    w = workloads.c6_seq_holes(scale=0.001)
    assert np.all(w.R[1:] > w.R[:-1])
    hits = np.isin(w.S, w.R)
    assert int(hits.sum()) == w.expected_count == int(round(len(w.S) * 0.9))
    # Misses are holes or above the largest key.
    assert not np.any(np.isin(w.S[~hits], w.R))
