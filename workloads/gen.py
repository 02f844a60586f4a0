"""Key generators on top of the counter-based draws in ``wl_gen.c``.

Every function is a pure function of its arguments and ``seed``: the same call
returns the same array on any machine and any thread count.  Sorting and
de-duplication use numpy (integer sorting has a unique result).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wl_gen.c")
_LIB = os.path.join(_HERE, "libwl.so")

# Stream labels: one sub-stream per purpose, so that changing one draw never
# shifts another.
LBL_R_POOL = 1
LBL_R_DROP = 2
LBL_HITS = 3
LBL_MISSES = 4
LBL_SHUFFLE = 5
LBL_RANK_PERM = 6
LBL_HOLES = 7
LBL_RUNS = 8


def build_lib(force: bool = False) -> str:
    """Compile ``wl_gen.c`` into ``libwl.so`` beside it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        L = ctypes.CDLL(_LIB)
        u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        vp = ctypes.c_void_p
        L.wl_stream_key.restype = u64
        L.wl_stream_key.argtypes = [u64, u64]
        L.wl_draw_u64.argtypes = [u64, u64, u64, u32, vp]
        L.wl_draw_range.argtypes = [u64, u64, u64, u64, u64, vp]
        L.wl_draw_bernoulli.argtypes = [u64, u64, u64, dbl, vp]
        L.wl_draw_lognormal.argtypes = [u64, u64, u64, dbl, dbl, vp]
        L.wl_scale_to_u63.argtypes = [vp, u64, dbl, vp]
        L.wl_draw_zipf1.argtypes = [u64, u64, u64, u64, vp]
        L.wl_permute.argtypes = [u64, u64, vp, u64, vp]
        L.wl_shuffle_u64.argtypes = [u64, vp, u64, vp]
        L.wl_floyd_mark.argtypes = [u64, u64, u64, vp]
        for f in ("wl_draw_u64", "wl_draw_range", "wl_draw_bernoulli",
                  "wl_draw_lognormal", "wl_scale_to_u63", "wl_draw_zipf1",
                  "wl_permute", "wl_shuffle_u64", "wl_floyd_mark"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def stream_key(seed: int, label: int) -> int:
    return int(lib().wl_stream_key(seed & (2**64 - 1), label))


def draw_u64(key: int, start: int, count: int, shift: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    if count:
        lib().wl_draw_u64(key, start, count, shift, _p(out))
    return out


def draw_range(key: int, start: int, count: int, lo: int, span: int) -> np.ndarray:
    assert span > 0
    out = np.empty(count, dtype=np.uint64)
    if count:
        lib().wl_draw_range(key, start, count, lo, span, _p(out))
    return out


def draw_bernoulli(key: int, start: int, count: int, p: float) -> np.ndarray:
    out = np.empty(count, dtype=np.uint8)
    if count:
        lib().wl_draw_bernoulli(key, start, count, p, _p(out))
    return out.view(bool)


def draw_zipf1(key: int, count: int, nmax: int) -> np.ndarray:
    """Ranks in [1, nmax] with P(k) proportional to 1/k."""
    out = np.empty(count, dtype=np.uint64)
    if count:
        lib().wl_draw_zipf1(key, 0, count, nmax, _p(out))
    return out


def permute(key: int, n: int, idx: np.ndarray) -> np.ndarray:
    """Apply the keyed bijection on [0, n) to every element of ``idx``."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty_like(idx)
    if len(idx):
        lib().wl_permute(key, n, _p(idx), len(idx), _p(out))
    return out


def shuffle(key: int, a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    if len(a):
        lib().wl_shuffle_u64(key, _p(a), len(a), _p(out))
    return out


def _sorted_unique(a: np.ndarray) -> np.ndarray:
    a = np.sort(a)
    if len(a) < 2:
        return a
    keep = np.empty(len(a), dtype=bool)
    keep[0] = True
    np.not_equal(a[1:], a[:-1], out=keep[1:])
    return a[keep]


def _unique_subset(draw_pool, n: int, seed: int) -> np.ndarray:
    """Draw pools of ceil(1.1 n) values until at least n distinct values are
    held, then drop a seeded random subset (Floyd) so exactly n remain."""
    pool = int(math.ceil(1.1 * n)) + 16
    acc = np.empty(0, dtype=np.uint64)
    start = 0
    while len(acc) < n:
        acc = _sorted_unique(np.concatenate([acc, draw_pool(start, pool)]))
        start += pool
    extra = len(acc) - n
    if extra:
        mark = np.zeros(len(acc), dtype=np.uint8)
        lib().wl_floyd_mark(stream_key(seed, LBL_R_DROP), len(acc), extra, _p(mark))
        acc = acc[mark == 0]
    return np.ascontiguousarray(acc)


def uniform_unique(n: int, bits: int, seed: int) -> np.ndarray:
    """n distinct keys uniform in [0, 2^bits), sorted (the ``unif`` shape)."""
    if n == 0:
        return np.empty(0, dtype=np.uint64)
    assert n <= 2**bits
    key = stream_key(seed, LBL_R_POOL)
    return _unique_subset(lambda s, c: draw_u64(key, s, c, 64 - bits), n, seed)


def lognormal_unique(n: int, sigma: float, seed: int, mu: float = 0.0) -> np.ndarray:
    """n distinct keys floor(v / v_max * 2^63) with v lognormal(mu, sigma) and
    v_max the largest value of the first pool, sorted (the ``lognorm``
    shape widened to 63 bits)."""
    if n == 0:
        return np.empty(0, dtype=np.uint64)
    key = stream_key(seed, LBL_R_POOL)
    state = {}

    def pool(start, count):
        v = np.empty(count, dtype=np.float64)
        lib().wl_draw_lognormal(key, start, count, mu, sigma, _p(v))
        if "vmax" not in state:
            state["vmax"] = float(v.max())
        out = np.empty(count, dtype=np.uint64)
        lib().wl_scale_to_u63(_p(v), count, state["vmax"], _p(out))
        return out

    return _unique_subset(pool, n, seed)


def seq_holes(n: int, seed: int, hole_p: float = 0.1) -> np.ndarray:
    """The first n values of 0, 1, 2, ... that survive independent deletion
    with probability ``hole_p`` (the ``seq_h`` shape), sorted and distinct."""
    if n == 0:
        return np.empty(0, dtype=np.uint64)
    key = stream_key(seed, LBL_HOLES)
    span = int(n / (1.0 - hole_p) * 1.05) + 64
    while True:
        deleted = draw_bernoulli(key, 0, span, hole_p)
        kept = np.flatnonzero(~deleted).astype(np.uint64)
        if len(kept) >= n:
            return np.ascontiguousarray(kept[:n])
        span *= 2


def dup_runs(rows: int, seed: int, max_run: int = 16, hole_p: float = 0.1) -> np.ndarray:
    """``seq_h`` values, each repeated U{1..max_run} times, until ``rows`` rows
    (the last run is truncated).  Sorted, with duplicates."""
    if rows == 0:
        return np.empty(0, dtype=np.uint64)
    rkey = stream_key(seed, LBL_RUNS)
    nvals = int(rows / ((1 + max_run) / 2.0) * 1.05) + 16
    while True:
        vals = seq_holes(nvals, seed, hole_p)
        reps = draw_range(rkey, 0, nvals, 1, max_run).astype(np.int64)
        total = int(reps.sum())
        if total >= rows:
            break
        nvals *= 2
    ends = np.cumsum(reps)
    last = int(np.searchsorted(ends, rows, side="left"))
    reps = reps[: last + 1].copy()
    reps[last] -= int(ends[last]) - rows
    out = np.repeat(vals[: last + 1], reps)
    assert len(out) == rows
    return np.ascontiguousarray(out)


def probe_mix(R: np.ndarray, m: int, hit_frac: float, seed: int, *,
              zipf_s: float | None = None, miss_lo: int = 0,
              miss_hi: int = 2**40) -> np.ndarray:
    """Outer keys: round(m*hit_frac) hits drawn with replacement from R's
    distinct keys (uniformly, or by Zipf(1) rank over a seeded scattering of
    ranks to keys), the rest uniform in [miss_lo, miss_hi) rejected until
    absent from R; then shuffled.  The number of hits is exact."""
    R = np.ascontiguousarray(R, dtype=np.uint64)
    distinct = _sorted_unique(R) if len(R) else R
    nd = len(distinct)
    n_hit = int(round(m * hit_frac)) if nd else 0
    n_miss = m - n_hit
    hkey = stream_key(seed, LBL_HITS)
    if n_hit:
        if zipf_s is None:
            pos = draw_range(hkey, 0, n_hit, 0, nd)
        else:
            assert zipf_s == 1.0, "only the exponent-1 Zipf law is generated"
            ranks = draw_zipf1(hkey, n_hit, nd)
            pos = permute(stream_key(seed, LBL_RANK_PERM), nd, ranks - np.uint64(1))
        hits = distinct[pos]
    else:
        hits = np.empty(0, dtype=np.uint64)
    mkey = stream_key(seed, LBL_MISSES)
    misses = []
    got, start = 0, 0
    while got < n_miss:
        want = int((n_miss - got) * 1.25) + 64
        cand = draw_range(mkey, start, want, miss_lo, miss_hi - miss_lo)
        start += want
        if nd:
            # Membership by binary search, queries in sorted order (random
            # queries into a large array miss the cache at every step).
            order = np.argsort(cand, kind="stable")
            j = np.empty(len(cand), dtype=np.int64)
            j[order] = np.searchsorted(distinct, cand[order])
            j[j >= nd] = nd - 1
            cand = cand[distinct[j] != cand]
        take = cand[: n_miss - got]
        misses.append(take)
        got += len(take)
    pre = np.concatenate([hits] + misses) if misses else hits
    return shuffle(stream_key(seed, LBL_SHUFFLE), pre)
