"""GPU parity: the HIP probe against the CPU oracle, bit-exact.

Every case builds the index through the C ABI, probes on the GPU and compares
the (s_idx, r_idx) pairs element by element with the oracle's sort-merge join
on the same seeded inputs (join output is integer index work: the bar is
exact equality, in the canonical (s_idx, r_idx) order).
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2111_08824_amd import lj

pytestmark = pytest.mark.gpu

U64MAX = 2**64 - 1
FLAGS = [lj.LJ_LEAF_FP32, lj.LJ_LEAF_FP64]
EXP = lj.LJ_SEARCH_EXPONENTIAL
BIN = lj.LJ_PROBE_BINNED
RADIX = lj.LJ_ROOT_RADIX
ALL_FLAGS = FLAGS + [lj.LJ_LEAF_FP32 | EXP, lj.LJ_LEAF_FP64 | EXP, lj.LJ_LEAF_FP32 | BIN,
                     lj.LJ_LEAF_FP64 | BIN, lj.LJ_LEAF_FP32 | EXP | BIN,
                     lj.LJ_LEAF_FP32 | RADIX, lj.LJ_LEAF_FP64 | RADIX,
                     lj.LJ_LEAF_FP32 | RADIX | BIN, lj.LJ_LEAF_FP32 | RADIX | EXP]


def gpu_join(R, S, leaves, flags, capacity=None):
    ix = lj.lj_build_rmi(np.asarray(R, dtype=np.uint64), leaves, flags)
    s = lj.to_device_keys(np.asarray(S, dtype=np.uint64))
    pairs = lj.probe(ix, s, capacity)
    out = pairs.cpu().numpy().view(np.uint32).reshape(-1, 2)
    return ix, out


def assert_parity(R, S, leaves, flags, label=""):
    print(f"[parity] {label} n={len(R)} m={len(S)} leaves={leaves} flags={flags}", flush=True)
    ix, got = gpu_join(R, S, leaves, flags)
    want = oracle.sort_merge_join(R, S)
    assert got.shape == want.shape, (got.shape, want.shape)
    assert np.array_equal(got, want)
    assert lj.lj_self_check(ix) == 0
    return got


@pytest.mark.parametrize("flags", ALL_FLAGS)
def test_uniform_1m(flags):
    w = workloads.c1_uniform()
    got = assert_parity(w.R, w.S, w.leaves, flags, w.name)
    assert len(got) == w.expected_count == 500_000


@pytest.mark.parametrize("flags", ALL_FLAGS)
def test_lognormal_zipf_2m(flags):
    w = workloads.c2_lognormal_zipf(scale=0.01)
    got = assert_parity(w.R, w.S, w.leaves, flags, w.name)
    assert len(got) == w.expected_count


@pytest.mark.parametrize("flags", ALL_FLAGS)
def test_dup_runs_1m(flags):
    w = workloads.c3_dup_runs(scale=0.01)
    assert_parity(w.R, w.S, w.leaves, flags, w.name)


@pytest.mark.parametrize("m", [1, 2, 63, 64, 255, 1023, 1024, 1025, 4096 + 7, 77_777])
@pytest.mark.parametrize("search", [0, EXP, BIN])
def test_ragged_tile_tails(m, search):
    R = workloads.gen.uniform_unique(50_000, 20, 3)
    S = workloads.gen.probe_mix(R, m, 0.6, 4, miss_hi=2**20)
    assert_parity(R, S, 256, lj.LJ_LEAF_FP32 | search, f"tail m={m}")


@pytest.mark.parametrize("leaves", [1, 2, 1000, 200_003])
@pytest.mark.parametrize("search", [0, EXP, BIN, RADIX, RADIX | BIN])
def test_leaf_counts(leaves, search):
    R = workloads.gen.lognormal_unique(50_000, 2.0, 5)
    S = workloads.gen.probe_mix(R, 60_000, 0.5, 6, miss_hi=2**63)
    assert_parity(R, S, leaves, lj.LJ_LEAF_FP32 | search, f"leaves={leaves}")


@pytest.mark.parametrize("flags", [lj.LJ_LEAF_FP32 | RADIX, lj.LJ_LEAF_FP32 | RADIX | BIN])
def test_radix_root_small_and_high_keys(flags):
    # Offsets from R[0] below 64 (their own root buckets), keys near 2^64
    # (the last buckets), outer keys below R[0] and above R[n-1].
    R = np.concatenate([np.arange(10, 90, dtype=np.uint64),
                        np.uint64(2**64 - 2**30) + np.arange(0, 3000, 7, dtype=np.uint64),
                        np.array([U64MAX], dtype=np.uint64)])
    S = np.concatenate([np.arange(0, 100, dtype=np.uint64), R[::3],
                        np.array([U64MAX, U64MAX - 1, 2**63], dtype=np.uint64)])
    for leaves in (1, 5, 64, 1000):
        assert_parity(R, S, leaves, flags, f"radix root small/high keys, leaves={leaves}")


def test_heavy_duplicates_load_balanced_emission():
    # One key repeated 5000 times in R and 3 times in S, other keys around it.
    R = np.concatenate([np.arange(0, 100, dtype=np.uint64),
                        np.full(5000, 1000, dtype=np.uint64),
                        np.arange(2000, 2100, dtype=np.uint64)])
    S = np.array([1000, 5, 1000, 7000, 2050, 1000], dtype=np.uint64)
    got = assert_parity(R, S, 8, lj.LJ_LEAF_FP32, "heavy duplicates")
    assert len(got) == 3 * 5000 + 2
    got = assert_parity(R, S, 8, lj.LJ_LEAF_FP32 | EXP, "heavy duplicates, exponential")
    assert len(got) == 3 * 5000 + 2
    got = assert_parity(R, S, 8, lj.LJ_LEAF_FP32 | BIN, "heavy duplicates, binned")
    assert len(got) == 3 * 5000 + 2


@pytest.mark.parametrize("flags", [lj.LJ_LEAF_FP64, lj.LJ_LEAF_FP64 | BIN])
def test_all_equal_inner_relation(flags):
    R = np.full(3000, 42, dtype=np.uint64)
    S = np.array([42, 41, 43, 42], dtype=np.uint64)
    got = assert_parity(R, S, 16, flags, "all equal")
    assert len(got) == 6000


@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097])
def test_binned_small_inner_relations(n):
    # Fewer keys in R than key ranges: most ranges are empty or share a fence.
    R = workloads.gen.uniform_unique(n, 24, 11)
    S = workloads.gen.probe_mix(R, 30_000, 0.7, 12, miss_hi=2**24)
    assert_parity(R, S, max(1, n // 64), lj.LJ_LEAF_FP32 | BIN, f"binned n={n}")


def test_extreme_keys():
    R = np.array([0, 0, 1, 2**63, U64MAX - 1, U64MAX, U64MAX], dtype=np.uint64)
    S = np.array([U64MAX, 0, 7, 2**63, U64MAX - 2, 1, U64MAX], dtype=np.uint64)
    for flags in ALL_FLAGS:
        assert_parity(R, S, 3, flags, "extreme keys")


@pytest.mark.parametrize("binned", [0, BIN])
def test_all_misses_and_empty_inputs(binned):
    R = workloads.gen.uniform_unique(10_000, 30, 8)
    S = np.array([2**40 + i for i in range(5000)], dtype=np.uint64)
    got = assert_parity(R, S, 64, lj.LJ_LEAF_FP32 | binned, "all misses")
    assert len(got) == 0
    # m = 0
    ix = lj.lj_build_rmi(R, 64, lj.LJ_LEAF_FP32 | binned)
    s0 = lj.to_device_keys(np.empty(0, dtype=np.uint64))
    assert lj.lj_probe_join(ix, s0) == (lj.LJ_OK, 0)
    # n = 0
    ix0 = lj.lj_build_rmi(np.empty(0, dtype=np.uint64), 4, lj.LJ_LEAF_FP32 | binned)
    s = lj.to_device_keys(np.array([0, 1, U64MAX], dtype=np.uint64))
    assert lj.lj_probe_join(ix0, s) == (lj.LJ_OK, 0)


@pytest.mark.parametrize("binned", [0, BIN])
def test_capacity_protocol(binned):
    import torch
    w = workloads.c3_dup_runs(scale=0.001)
    want = oracle.sort_merge_join(w.R, w.S)
    ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32 | binned)
    s = lj.to_device_keys(w.S)
    st, cnt = lj.lj_probe_join(ix, s, None)  # count only
    assert (st, cnt) == (lj.LJ_OK, len(want))
    cap = len(want) // 3
    out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    st, cnt = lj.lj_probe_join(ix, s, out)
    assert st == lj.LJ_ERR_CAPACITY and cnt == len(want)
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want[:cap])  # the first cap pairs, in order


@pytest.mark.parametrize("binned", [0, BIN])
def test_split_invariance(binned):
    w = workloads.c2_lognormal_zipf(scale=0.005)
    ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32 | binned)
    whole = lj.probe(ix, lj.to_device_keys(w.S)).cpu().numpy().view(np.uint32)
    parts = []
    cuts = [0, 1, 1000, 1024 * 7 + 3, 400_000, len(w.S)]
    for a, b in zip(cuts[:-1], cuts[1:]):
        p = lj.probe(ix, lj.to_device_keys(w.S[a:b])).cpu().numpy().view(np.uint32).copy()
        p[:, 0] += a
        parts.append(p)
    assert np.array_equal(np.concatenate(parts), whole)


@pytest.mark.parametrize("binned", [0, BIN])
def test_async_matches_sync_and_checks_workspace(binned):
    import torch
    w = workloads.c1_uniform(scale=0.2)
    want = oracle.sort_merge_join(w.R, w.S)
    ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32 | binned)
    s = lj.to_device_keys(w.S)
    nbytes = lj.lj_probe_workspace_bytes(ix, len(w.S))
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty((len(want) + 5, 2), dtype=torch.int32, device="cuda")
    for _ in range(3):  # the workspace is reused across calls
        lj.lj_probe_join_async(ix, s, out, cnt, ws)
        torch.cuda.synchronize()
        assert int(cnt.item()) == len(want)
        assert np.array_equal(out[: len(want)].cpu().numpy().view(np.uint32), want)
    small = torch.empty(4, dtype=torch.int64, device="cuda")
    with pytest.raises(lj.LJError) as e:
        lj.lj_probe_join_async(ix, s, out, cnt, small)
    assert e.value.status == lj.LJ_ERR_WORKSPACE


def test_device_windows_equal_host_windows():
    import torch
    for w in (workloads.c1_uniform(scale=0.1), workloads.c2_lognormal_zipf(scale=0.002)):
        for flags in FLAGS + [lj.LJ_LEAF_FP32 | RADIX, lj.LJ_LEAF_FP64 | RADIX]:
            ix = lj.lj_build_rmi(w.R, w.leaves, flags)
            keys = np.concatenate([w.R, w.S])
            leaf_h, pred_h, lo_h, hi_h = lj.lj_predict_windows_host(ix, keys)
            kd = lj.to_device_keys(keys)
            leaf = torch.empty(len(keys), dtype=torch.int32, device="cuda")
            pred = torch.empty(len(keys), dtype=torch.int64, device="cuda")
            lo = torch.empty(len(keys), dtype=torch.int64, device="cuda")
            hi = torch.empty(len(keys), dtype=torch.int64, device="cuda")
            lj.lj_predict_windows(ix, kd, leaf, pred, lo, hi)
            torch.cuda.synchronize()
            assert np.array_equal(leaf.cpu().numpy().view(np.uint32), leaf_h)
            assert np.array_equal(pred.cpu().numpy(), pred_h)
            assert np.array_equal(lo.cpu().numpy(), lo_h)
            assert np.array_equal(hi.cpu().numpy(), hi_h)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 31, 32, 33, 1000])
def test_windows_around_line_boundaries(n):
    # The binary search reads one key per 16-key line of R first, then the
    # candidate positions inside one line: every key of R, every gap
    # between keys and both ends, with one leaf (window = all of R) and
    # many, and FP32 / FP64 leaves.
    R = np.arange(0, 3 * n, 3, dtype=np.uint64) + np.uint64(5)
    S = np.arange(0, 3 * n + 9, dtype=np.uint64)
    for leaves in (1, max(1, n // 4)):
        for flags in FLAGS + [lj.LJ_LEAF_FP32 | BIN, lj.LJ_LEAF_FP32 | RADIX]:
            assert_parity(R, S, leaves, flags, f"line boundaries n={n}")
    D = np.repeat(R, 3)  # runs of three equal keys across line ends
    assert_parity(D, S, 1, lj.LJ_LEAF_FP32, f"line boundaries dup n={n}")


@pytest.mark.parametrize("binned", [0, BIN])
def test_radix_root_clusters_big_leaves_and_runs(binned):
    # Radix root on: (1) clusters of keys a few apart spread over [0, 2^60)
    # (many keys share a root bucket's interpolation); (2) one key repeated
    # 600 times beside ordinary keys (one leaf far larger than the rest);
    # (3) runs of equal keys across line ends.
    rng = np.random.default_rng(77)
    base = np.sort(rng.choice(2**60, 3000, replace=False).astype(np.uint64))
    R1 = np.unique(np.concatenate([base + np.uint64(j) for j in range(0, 40, 3)]))
    S1 = np.concatenate([R1[::5], R1[::7] + np.uint64(1), base - np.uint64(1),
                         rng.integers(0, 2**60, 20_000, dtype=np.uint64)])
    R2 = np.sort(np.concatenate([workloads.gen.uniform_unique(100_000, 40, 5),
                                 np.full(600, 2**39 + 12345, dtype=np.uint64)]))
    S2 = np.concatenate([R2[::3], np.full(50, 2**39 + 12345, dtype=np.uint64),
                         rng.integers(0, 2**40, 30_000, dtype=np.uint64)])
    R3 = np.repeat(np.arange(0, 30_000, 2, dtype=np.uint64), 5)  # runs of 5 across lines
    S3 = np.arange(0, 30_010, dtype=np.uint64)
    for R, S, label in ((R1, S1, "ties"), (R2, S2, "big leaf"), (R3, S3, "runs")):
        for leaves in (max(1, len(R) // 200), max(1, len(R) // 50)):
            assert_parity(R, S, leaves, lj.LJ_LEAF_FP32 | RADIX | binned,
                          f"radix root: {label}, leaves={leaves}")
