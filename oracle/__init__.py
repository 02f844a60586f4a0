"""CPU oracle for the learned indexed nested loop join -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

The join result has a plain definition (Section II-A, INLJ; Section VI-B,
"Duplicates"): given R non-decreasing and S arbitrary,

    P = {(i, j) : S[i] == R[j]}  in lexicographic (i, j) order,  count = |P|.

The learned index (Section II-D, RMI; Section III) only changes how fast P is
found, never P itself.  The learned sort join (Section IV) takes R in any
order; its P is the same with j the position in R as given (``sort_join``),
and its sorted relations are the (key, position) order (``sort_positions``).  ``oracle.c`` computes P three independent ways; see
its header.  Parity of the model parameters themselves (slopes, intercepts,
bound widths) is unpinned: the paper prints no values for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build_lib(force: bool = False) -> str:
    """Compile ``oracle.c`` (plain C, -O2, no fast-math) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        L = ctypes.CDLL(_LIB)
        vp, u64 = ctypes.c_void_p, ctypes.c_uint64
        pp = ctypes.POINTER(ctypes.c_void_p)
        cp = ctypes.POINTER(ctypes.c_uint64)
        L.orc_is_nondecreasing.argtypes = [vp, u64]
        L.orc_is_nondecreasing.restype = ctypes.c_int
        L.orc_sort_positions.argtypes = [vp, u64, vp, vp]
        L.orc_sort_positions.restype = ctypes.c_int
        for f in (L.orc_brute_join, L.orc_sort_merge_join, L.orc_sort_join):
            f.argtypes = [vp, u64, vp, u64, pp, cp]
            f.restype = ctypes.c_int
        L.orc_equal_range.argtypes = [vp, u64, vp, u64, vp, vp]
        L.orc_equal_range.restype = None
        L.orc_free.argtypes = [vp]
        L.orc_free.restype = None
        _lib = L
    return _lib


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


def is_nondecreasing(R) -> bool:
    R = _u64(R)
    return bool(_L().orc_is_nondecreasing(R.ctypes.data, len(R)))


def _join(fn, R, S) -> np.ndarray:
    R, S = _u64(R), _u64(S)
    ptr = ctypes.c_void_p()
    cnt = ctypes.c_uint64()
    rc = fn(R.ctypes.data, len(R), S.ctypes.data, len(S), ctypes.byref(ptr),
            ctypes.byref(cnt))
    if rc == -2:
        raise ValueError("R is not non-decreasing")
    if rc != 0:
        raise MemoryError("oracle join ran out of host memory")
    k = cnt.value
    try:
        if k == 0:
            return np.empty((0, 2), dtype=np.uint32)
        buf = (ctypes.c_uint32 * (2 * k)).from_address(ptr.value)
        return np.frombuffer(buf, dtype=np.uint32).reshape(k, 2).copy()
    finally:
        if ptr.value:
            _L().orc_free(ptr)


def brute_join(R, S) -> np.ndarray:
    """(k, 2) uint32 array of (s_idx, r_idx) pairs by nested loops."""
    return _join(_L().orc_brute_join, R, S)


def sort_merge_join(R, S) -> np.ndarray:
    """(k, 2) uint32 array of (s_idx, r_idx) pairs by sort-merge."""
    return _join(_L().orc_sort_merge_join, R, S)


def sort_join(R, S) -> np.ndarray:
    """(k, 2) uint32 array of (s_idx, r_idx) pairs for R in any order
    (r_idx = position in R as given), by sorting both sides and merging."""
    return _join(_L().orc_sort_join, R, S)


def sort_positions(keys):
    """(sorted keys, input positions) in ascending (key, position) order."""
    keys = _u64(keys)
    out_k = np.empty(len(keys), dtype=np.uint64)
    out_p = np.empty(len(keys), dtype=np.uint32)
    if len(keys) and _L().orc_sort_positions(keys.ctypes.data, len(keys), out_k.ctypes.data,
                                             out_p.ctypes.data):
        raise MemoryError("oracle sort ran out of host memory")
    return out_k, out_p


def equal_range(R, keys):
    """(first, count) arrays: the run of sorted R equal to each key."""
    R, keys = _u64(R), _u64(keys)
    first = np.empty(len(keys), dtype=np.uint64)
    count = np.empty(len(keys), dtype=np.uint64)
    if len(keys):
        _L().orc_equal_range(R.ctypes.data, len(R), keys.ctypes.data, len(keys),
                             first.ctypes.data, count.ctypes.data)
    return first, count
