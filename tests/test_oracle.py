"""Pins for the CPU oracle (no GPU).

The join result is P = {(i, j) : S[i] == R[j]} in (i, j) order (Section II-A,
INLJ; Section VI-B, "Duplicates").  The sort-merge oracle is pinned against:
  * the definition written as nested loops (brute force), exhaustively on
    tiny domains and on random small cases with heavy duplication;
  * the closed-form count |P| = sum_k mult_R(k) * mult_S(k), computed with a
    Python Counter that shares nothing with the merge;
  * structural facts of P: every pair matches, (i, j) order is strict,
    each i's r indices form one contiguous run of R;
  * the generator's exact hit count on the uniform 1M workload;
  * planted mistakes: mutated copies of oracle.c must fail these pins.
"""
import collections
import itertools
import os
import shutil
import subprocess
import ctypes

import numpy as np
import pytest

import oracle
import workloads

U64MAX = 2**64 - 1


def count_invariant(R, S) -> int:
    cr = collections.Counter(int(x) for x in R)
    cs = collections.Counter(int(x) for x in S)
    return sum(cr[k] * v for k, v in cs.items())


def check_structure(R, S, P):
    R = np.asarray(R, dtype=np.uint64)
    S = np.asarray(S, dtype=np.uint64)
    if len(P) == 0:
        return
    i, j = P[:, 0].astype(np.int64), P[:, 1].astype(np.int64)
    assert np.all(S[i] == R[j]), "pair with unequal keys"
    key = i * (len(R) + 1) + j
    assert np.all(np.diff(key) > 0), "pairs not in strict (i, j) order"


def test_hand_example():
    # R has a duplicate run; S repeats a key and contains keys absent from R
    # (below, between and above R's keys).
    R = [1, 3, 3, 5, 9]
    S = [3, 4, 9, 3, 0, 1, 10]
    want = [[0, 1], [0, 2], [2, 4], [3, 1], [3, 2], [5, 0]]
    assert oracle.brute_join(R, S).tolist() == want
    assert oracle.sort_merge_join(R, S).tolist() == want


def test_empty_relations():
    e = np.empty(0, dtype=np.uint64)
    one = np.array([7], dtype=np.uint64)
    for R, S in [(e, e), (e, one), (one, e)]:
        assert oracle.sort_merge_join(R, S).shape == (0, 2)
        assert oracle.brute_join(R, S).shape == (0, 2)


def test_extreme_keys():
    R = np.array([0, 0, 2**63, U64MAX, U64MAX], dtype=np.uint64)
    S = np.array([U64MAX, 0, U64MAX - 1, 2**63, 1], dtype=np.uint64)
    want = [[0, 3], [0, 4], [1, 0], [1, 1], [3, 2]]
    assert oracle.sort_merge_join(R, S).tolist() == want
    assert oracle.brute_join(R, S).tolist() == want


def test_unsorted_r_rejected():
    assert not oracle.is_nondecreasing([3, 2])
    assert oracle.is_nondecreasing([2, 2, 3])
    with pytest.raises(ValueError):
        oracle.sort_merge_join([3, 2], [2])


def test_exhaustive_tiny_domain():
    # Every R (non-decreasing, length <= 4, keys in {0,1,2}) against every S
    # of length <= 3 over {0,1,2,3}.
    for n in range(0, 5):
        for R in itertools.combinations_with_replacement(range(3), n):
            for m in range(0, 4):
                for S in itertools.product(range(4), repeat=m):
                    a = oracle.sort_merge_join(R, S)
                    b = oracle.brute_join(R, S)
                    assert a.tolist() == b.tolist(), (R, S)
                    assert len(a) == count_invariant(R, S)


@pytest.mark.parametrize("seed", range(40))
def test_random_small_vs_brute(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 400))
    m = int(rng.integers(0, 400))
    dom = int(rng.choice([2, 8, 64, 1000, 2**40]))
    R = np.sort(rng.integers(0, dom, n, dtype=np.uint64))
    S = rng.integers(0, dom, m, dtype=np.uint64)
    a = oracle.sort_merge_join(R, S)
    b = oracle.brute_join(R, S)
    assert np.array_equal(a, b)
    assert len(a) == count_invariant(R, S)
    check_structure(R, S, a)


def test_equal_range_vs_scan():
    rng = np.random.default_rng(5)
    R = np.sort(rng.integers(0, 50, 300, dtype=np.uint64))
    q = np.concatenate([np.arange(0, 52, dtype=np.uint64),
                        np.array([U64MAX], dtype=np.uint64)])
    first, count = oracle.equal_range(R, q)
    for t, key in enumerate(q):
        hits = np.flatnonzero(R == key)
        assert count[t] == len(hits)
        if len(hits):
            assert first[t] == hits[0]
            assert hits[-1] - hits[0] + 1 == len(hits)
        else:
            assert first[t] == np.searchsorted(R, key, side="left")


def test_uniform_1m_exact_hits():
    # The uniform 1M workload draws exactly 500,000 hits against a unique R
    # and rejects every miss present in R, so |P| = 500,000.
    w = workloads.c1_uniform()
    P = oracle.sort_merge_join(w.R, w.S)
    assert len(P) == w.expected_count == 500_000
    check_structure(w.R, w.S, P)
    # every s index appears at most once (R is unique)
    assert len(np.unique(P[:, 0])) == len(P)


def test_dup_runs_count_invariant():
    w = workloads.c3_dup_runs(scale=0.001)
    P = oracle.sort_merge_join(w.R, w.S)
    ur, cr = np.unique(w.R, return_counts=True)
    us, cs = np.unique(w.S, return_counts=True)
    common, ir, is_ = np.intersect1d(ur, us, assume_unique=True, return_indices=True)
    assert len(P) == int(np.sum(cr[ir].astype(np.int64) * cs[is_].astype(np.int64)))
    check_structure(w.R, w.S, P)


# --- planted mistakes: each mutant of oracle.c must fail the pins above ----

MUTANTS = {
    "merge-advances-wrong-side": ("if (T[a].key < R[b]) {", "if (T[a].key <= R[b]) {"),
    "run-truncated": ("while (b2 < n && R[b2] == key) ++b2;", "b2 = b + 1;"),
    "no-final-sort": ("sorted[2 * dst] = v.p[2 * k];", "sorted[2 * k] = v.p[2 * k];"
                      " (void)dst;"),
    "upper-bound-off": ("if (R[mid] <= q) lo2 = mid + 1;", "if (R[mid] < q) lo2 = mid + 1;"),
    "s-run-truncated": ("while (a2 < m && T[a2].key == key) ++a2;", "a2 = a + 1;"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert old in src, name
    if name == "no-final-sort":
        src = src.replace("sorted[2 * dst + 1] = v.p[2 * k + 1];",
                          "sorted[2 * k + 1] = v.p[2 * k + 1];")
    src = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-w", "-o", str(so), str(c)],
                   check=True)
    return ctypes.CDLL(str(so))


def _pins_hold(L) -> bool:
    """Rerun the core pins against a library built from oracle.c text."""
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    L.orc_sort_merge_join.argtypes = [vp, u64, vp, u64, ctypes.POINTER(vp),
                                      ctypes.POINTER(u64)]
    L.orc_equal_range.argtypes = [vp, u64, vp, u64, vp, vp]
    rng = np.random.default_rng(11)
    for _ in range(30):
        R = np.sort(rng.integers(0, 6, int(rng.integers(1, 30)), dtype=np.uint64))
        S = rng.integers(0, 7, int(rng.integers(1, 30)), dtype=np.uint64)
        ptr, cnt = vp(), u64()
        L.orc_sort_merge_join(R.ctypes.data, len(R), S.ctypes.data, len(S),
                              ctypes.byref(ptr), ctypes.byref(cnt))
        k = cnt.value
        got = (np.frombuffer((ctypes.c_uint32 * (2 * k)).from_address(ptr.value),
                             dtype=np.uint32).reshape(k, 2).tolist() if k else [])
        if got != oracle.brute_join(R, S).tolist() or k != count_invariant(R, S):
            return False
        q = np.arange(8, dtype=np.uint64)
        first = np.empty(8, dtype=np.uint64)
        count = np.empty(8, dtype=np.uint64)
        L.orc_equal_range(R.ctypes.data, len(R), q.ctypes.data, 8, first.ctypes.data,
                          count.ctypes.data)
        if any(int(count[t]) != int(np.sum(R == q[t])) for t in range(8)):
            return False
    return True


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_unmutated_copy_passes(tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    c = tmp_path / "orig.c"
    c.write_text(src)
    so = tmp_path / "orig.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), str(c)], check=True)
    assert _pins_hold(ctypes.CDLL(str(so)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    assert not _pins_hold(_build_mutant(tmp_path, name))
