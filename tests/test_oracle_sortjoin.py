"""Pins for the oracle of the learned sort join (Section IV), no GPU.

The learned sort join takes R in any order.  Its result is the join's plain
definition P = {(i, j) : S[i] == R[j]} in (i, j) order with j the position
in R as given, and its sort phase leaves each relation in (key, position)
order.  ``oracle.sort_join`` and ``oracle.sort_positions`` are pinned
against:
  * nested loops (``oracle.brute_join``, which reads R in any order),
    exhaustively on tiny domains and on random cases with heavy duplication;
  * the closed-form count sum_k mult_R(k) * mult_S(k) (Python Counter);
  * the sort-merge oracle of a sorted R after mapping its positions through
    the sorting permutation;
  * Python's own sort of (key, position) tuples;
  * planted mistakes: mutated copies of oracle.c must fail these pins.
"""
import collections
import ctypes
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

U64MAX = 2**64 - 1


def count_invariant(R, S) -> int:
    cr = collections.Counter(int(x) for x in R)
    return sum(cr[int(x)] for x in S)


def test_hand_example():
    # R unsorted with a duplicate; S hits, misses and repeats.
    R = [30, 10, 30, 20]
    S = [30, 20, 99, 10, 30]
    want = [[0, 0], [0, 2], [1, 3], [3, 1], [4, 0], [4, 2]]
    assert oracle.sort_join(R, S).tolist() == want
    k, p = oracle.sort_positions(R)
    assert k.tolist() == [10, 20, 30, 30] and p.tolist() == [1, 3, 0, 2]


def test_empty_and_extreme():
    assert oracle.sort_join([], [1, 2]).shape == (0, 2)
    assert oracle.sort_join([1, 2], []).shape == (0, 2)
    R = [U64MAX, 0, U64MAX, 1, 0]
    S = [0, U64MAX, 2, 1]
    assert oracle.sort_join(R, S).tolist() == oracle.brute_join(R, S).tolist()
    k, p = oracle.sort_positions(R)
    assert k.tolist() == [0, 0, 1, U64MAX, U64MAX] and p.tolist() == [1, 4, 3, 0, 2]


def test_exhaustive_tiny_domain():
    for nr in range(4):
        for R in itertools.product(range(3), repeat=nr):
            for S in itertools.product(range(4), repeat=3):
                got = oracle.sort_join(R, S).tolist()
                assert got == oracle.brute_join(R, S).tolist(), (R, S)


@pytest.mark.parametrize("seed", range(6))
def test_random_vs_brute(seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        n, m = int(rng.integers(0, 200)), int(rng.integers(0, 200))
        dom = int(rng.integers(1, 60))
        R = rng.integers(0, dom, n, dtype=np.uint64)
        S = rng.integers(0, dom + 5, m, dtype=np.uint64)
        P = oracle.sort_join(R, S)
        assert P.tolist() == oracle.brute_join(R, S).tolist()
        assert len(P) == count_invariant(R, S)


def test_matches_sort_merge_after_permutation():
    rng = np.random.default_rng(5)
    R = rng.integers(0, 5000, 20000, dtype=np.uint64)
    S = rng.integers(0, 6000, 15000, dtype=np.uint64)
    sk, sp = oracle.sort_positions(R)
    P_sorted = oracle.sort_merge_join(sk, S)
    mapped = np.stack([P_sorted[:, 0], sp[P_sorted[:, 1]]], axis=1)
    # Positions of equal keys ascend in sp, so the mapped pairs keep (i, j) order.
    assert np.array_equal(oracle.sort_join(R, S), mapped)
    assert len(mapped) == count_invariant(R, S)


def test_sort_positions_vs_python_sort():
    rng = np.random.default_rng(9)
    for n in (0, 1, 2, 17, 1000):
        keys = rng.integers(0, max(1, n // 3), n, dtype=np.uint64)
        keys[: n // 10] = U64MAX
        k, p = oracle.sort_positions(keys)
        want = sorted(zip(keys.tolist(), range(n)))
        assert k.tolist() == [a for a, _ in want]
        assert p.tolist() == [b for _, b in want]


# --- planted mistakes in the sort join's code paths ----------------------

MUTANTS = {
    "merge-advances-wrong-side": ("if (T[a].key < U[b].key) {", "if (T[a].key <= U[b].key) {"),
    "r-run-truncated": ("while (b2 < n && U[b2].key == key) ++b2;", "b2 = b + 1;"),
    "r-position-not-mapped": ("push(&v, T[k].idx, U[l].idx)", "push(&v, T[k].idx, l)"),
    "positions-not-carried": ("out_pos[j] = (uint32_t)T[j].idx;", "out_pos[j] = (uint32_t)j;"),
}


def _pins_hold(L) -> bool:
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    L.orc_sort_join.argtypes = [vp, u64, vp, u64, ctypes.POINTER(vp), ctypes.POINTER(u64)]
    L.orc_sort_positions.argtypes = [vp, u64, vp, vp]
    rng = np.random.default_rng(13)
    for _ in range(30):
        R = rng.integers(0, 6, int(rng.integers(1, 30)), dtype=np.uint64)
        S = rng.integers(0, 7, int(rng.integers(1, 30)), dtype=np.uint64)
        ptr, cnt = vp(), u64()
        L.orc_sort_join(R.ctypes.data, len(R), S.ctypes.data, len(S), ctypes.byref(ptr),
                        ctypes.byref(cnt))
        k = cnt.value
        got = (np.frombuffer((ctypes.c_uint32 * (2 * k)).from_address(ptr.value),
                             dtype=np.uint32).reshape(k, 2).tolist() if k else [])
        if got != oracle.brute_join(R, S).tolist():
            return False
        sk = np.empty(len(R), dtype=np.uint64)
        sp = np.empty(len(R), dtype=np.uint32)
        L.orc_sort_positions(R.ctypes.data, len(R), sk.ctypes.data, sp.ctypes.data)
        want = sorted(zip(R.tolist(), range(len(R))))
        if sk.tolist() != [a for a, _ in want] or sp.tolist() != [b for _, b in want]:
            return False
    return True


def _build(tmp_path, name, src):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-w", "-o", str(so), str(c)], check=True)
    return ctypes.CDLL(str(so))


def _source():
    return open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_unmutated_copy_passes(tmp_path):
    assert _pins_hold(_build(tmp_path, "orig", _source()))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = _source()
    assert src.count(old) == 1, name
    assert not _pins_hold(_build(tmp_path, name, src.replace(old, new)))
