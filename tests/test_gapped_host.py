"""Host checks of the gapped RMI build (Section III-A, "GRMI Building" and
"GRMI Lookup"), no GPU needed.

The slot arrays of a host-only gapped index are read back and checked
against what model-based insertion must produce, independently of the build
code: R's keys in order, each exactly once with its own position as payload,
every gap holding the next key, each key inside the slot window a probe of it
searches; and, against the oracle's equal_range, that the lower bound of
every probe key among the slots from its predicted slot on is the slot of its
first copy in R and lies inside its window, so the probe's forward search
finds exactly the oracle's run.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2111_08824_amd import lj

U64MAX = 2**64 - 1


def slots_of(R, leaves, spk, flags=lj.LJ_LEAF_FP32):
    ix = lj.lj_build_gapped_rmi_host_only(np.asarray(R, dtype=np.uint64), leaves, spk, flags)
    keys, ridx = lj.lj_gapped_slots_host(ix)
    return ix, keys, ridx


def check_slots(R, leaves, spk, flags=lj.LJ_LEAF_FP32):
    R = np.asarray(R, dtype=np.uint64)
    ix, keys, ridx = slots_of(R, leaves, spk, flags)
    st = ix.stats
    n = len(R)
    assert st.slots_per_key == spk and st.nslots == len(keys)
    assert len(keys) >= max(1, n * spk)
    real = ridx != lj.GAP_SLOT
    # R in order, each position once, with its own key.
    assert np.array_equal(ridx[real], np.arange(n, dtype=np.uint32))
    assert np.array_equal(keys[real], R)
    # A gap holds the key of the next key slot (UINT64_MAX after the last).
    j = np.arange(len(keys))
    nxt = np.searchsorted(np.flatnonzero(real), j, side="left")
    after = np.append(R, np.uint64(U64MAX))
    assert np.array_equal(keys[~real], after[nxt[~real]])
    # So the key array is non-decreasing.
    assert np.all(keys[1:] >= keys[:-1])
    # Equal keys sit in adjacent slots.
    pos = np.flatnonzero(real)
    same = R[1:] == R[:-1]
    assert np.all(pos[1:][same] == pos[:-1][same] + 1)
    # Every key lies in the slot window [pred, pred + drift] of its leaf.
    if n:
        _, pred, lo, hi = lj.lj_predict_windows_host(ix, R)
        assert np.all(lo == pred)
        assert np.all((lo <= pos) & (pos <= hi))
    return ix, keys, ridx


@pytest.mark.parametrize("spk", [1, 2, 4, 9])
@pytest.mark.parametrize("flags", [lj.LJ_LEAF_FP32, lj.LJ_LEAF_FP64])
def test_slots_of_workloads(spk, flags):
    for R, leaves in ((workloads.c1_uniform(scale=0.1).R, 1000),
                      (workloads.c2_lognormal_zipf(scale=0.002).R, 2048),
                      (workloads.c3_dup_runs(scale=0.002).R, 500),
                      (workloads.gen.seq_holes(100_000, 9), 300)):
        check_slots(R, leaves, spk, flags)


def test_slot_windows_find_the_oracle_run():
    for w in (workloads.c2_lognormal_zipf(scale=0.002), workloads.c3_dup_runs(scale=0.002)):
        ix, keys, ridx = check_slots(w.R, w.leaves, 4)
        _, pred, lo, hi = lj.lj_predict_windows_host(ix, w.S)
        first, count = oracle.equal_range(w.R, w.S)
        hit = count > 0
        assert 0 < hit.sum() < len(w.S)
        # Lower bound of each key among the slots from its predicted slot on
        # (gaps before the first copy can hold the key too).
        lb = np.searchsorted(keys, w.S, side="left")
        lb[hit] = np.maximum(lb[hit], lo[hit])
        # Hits: that is the key slot of the first copy, inside the window,
        # followed by the other copies.
        assert np.all(lb[hit] <= hi[hit])
        assert np.array_equal(ridx[lb[hit]].astype(np.int64), first[hit].astype(np.int64))
        last = lb[hit] + count[hit].astype(np.int64) - 1
        assert np.array_equal(ridx[last].astype(np.int64),
                              (first[hit] + count[hit] - 1).astype(np.int64))
        # Misses: no key slot holds the key.
        in_range = lb[~hit] < len(keys)
        lbm = lb[~hit][in_range]
        assert not np.any((keys[lbm] == w.S[~hit][in_range]) & (ridx[lbm] != lj.GAP_SLOT))


def test_more_slots_per_key_shrink_the_drift():
    R = workloads.c2_lognormal_zipf(scale=0.005).R
    d1 = lj.lj_build_gapped_rmi_host_only(R, 4096, 1).stats.mean_window
    d4 = lj.lj_build_gapped_rmi_host_only(R, 4096, 4).stats.mean_window
    d16 = lj.lj_build_gapped_rmi_host_only(R, 4096, 16).stats.mean_window
    assert d16 <= d4 <= d1


def test_extreme_and_degenerate_relations():
    for R in ([0, 0, 1, 2**63, U64MAX - 1, U64MAX, U64MAX], [5], [7] * 1000, [U64MAX] * 3,
              list(range(100))):
        for leaves in (1, 3, 64):
            check_slots(R, leaves, 4)
    ix, keys, ridx = slots_of(np.empty(0, dtype=np.uint64), 8, 4)
    assert len(keys) == 1 and ridx[0] == lj.GAP_SLOT and keys[0] == np.uint64(U64MAX)


def test_gapped_build_arguments():
    R = np.arange(100, dtype=np.uint64)
    for bad in (0, 17):
        with pytest.raises(lj.LJError) as e:
            lj.lj_build_gapped_rmi_host_only(R, 4, bad)
        assert e.value.status == lj.LJ_ERR_ARG
    plain = lj.lj_build_rmi_host_only(R, 4)
    assert plain.stats.slots_per_key == 0 and plain.stats.nslots == 0
    with pytest.raises(lj.LJError) as e:
        lj.lj_gapped_slots_host(plain)
    assert e.value.status == lj.LJ_ERR_ARG
    unsorted = np.array([3, 1, 2], dtype=np.uint64)
    with pytest.raises(lj.LJError) as e:
        lj.lj_build_gapped_rmi_host_only(unsorted, 4, 4)
    assert e.value.status == lj.LJ_ERR_UNSORTED
