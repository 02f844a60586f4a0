"""Expected join output for a duplicate-free sorted R, from the oracle.

When R has no duplicate keys, P = {(i, j) : S[i] == R[j]} holds exactly one
pair per outer key that occurs in R, with j its position, so the oracle's
textbook equal_range (lower and upper bound by binary search) gives P element
by element: (i, first_i) for every i with count_i == 1.  The searches of
independent slices of S run in host threads (the oracle's C routine releases
the interpreter lock), which is what makes this affordable for 1e8 keys.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

HOST_THREADS = max(1, min(16, os.cpu_count() or 1))


def equal_range_threaded(R: np.ndarray, keys: np.ndarray, threads: int = HOST_THREADS):
    """oracle.equal_range over slices of `keys` in parallel threads."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    if len(keys) < 1 << 16 or threads == 1:
        return oracle.equal_range(R, keys)
    cuts = np.linspace(0, len(keys), threads + 1).astype(np.int64)
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda ab: oracle.equal_range(R, keys[ab[0]:ab[1]]),
                            zip(cuts[:-1], cuts[1:])))
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))


def expected_pairs_unique(R: np.ndarray, S: np.ndarray, threads: int = HOST_THREADS) -> np.ndarray:
    """(k, 2) uint32 array of P for a duplicate-free sorted R."""
    first, count = equal_range_threaded(R, S, threads)
    assert np.all(count <= 1), "R has duplicate keys"
    hit = np.flatnonzero(count == 1)
    out = np.empty((len(hit), 2), dtype=np.uint32)
    out[:, 0] = hit
    out[:, 1] = first[hit]
    return out
