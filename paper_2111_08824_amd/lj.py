"""Python binding of the C ABI in include/lj.h (argument marshalling only).

Every step of the probe runs in the HIP kernels of liblj.so; this module only
converts numpy arrays and torch tensors to pointers and sizes.  It fails
loudly when liblj.so has not been built: there is no fallback path.

Memory conventions: R is passed as a host numpy array (the index uploads its
own copy); S, the output pairs and device counters are torch CUDA tensors,
with uint64 keys carried in int64 tensors (bit-identical storage).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblj.so")

LJ_OK = 0
LJ_ERR_ARG = -1
LJ_ERR_UNSORTED = -2
LJ_ERR_TOO_LARGE = -3
LJ_ERR_CAPACITY = -4
LJ_ERR_DEVICE = -5
LJ_ERR_OOM = -6
LJ_ERR_WORKSPACE = -7
LJ_ERR_TIMEOUT = -8

LJ_LEAF_FP32 = 1
LJ_LEAF_FP64 = 2
LJ_SEARCH_EXPONENTIAL = 4
LJ_PROBE_BINNED = 8
LJ_ROOT_RADIX = 16

EXPORTED = (
    "lj_build_rmi", "lj_free_index", "lj_probe_join", "lj_probe_workspace_bytes",
    "lj_probe_join_async", "lj_index_get_stats", "lj_self_check", "lj_predict_windows",
    "lj_predict_windows_host", "lj_build_rmi_host_only", "lj_probe_set_timing_events",
    "lj_bench_random_gather", "lj_strerror", "lj_batch_default_tuning",
    "lj_batch_plan_create", "lj_batch_plan_run", "lj_batch_plan_destroy", "lj_batch_autotune",
    "lj_server_default_config", "lj_server_create", "lj_server_submit",
    "lj_server_submit_device", "lj_server_wait", "lj_server_replay", "lj_server_get_stats",
    "lj_server_destroy",
    "lj_build_gapped_rmi", "lj_build_gapped_rmi_host_only", "lj_gapped_slots_host",
    "lj_build_learned_hash", "lj_build_learned_hash_host_only", "lj_hash_buckets_host",
    "lj_sort_join_workspace_bytes", "lj_sort_join_async", "lj_learned_sort_async",
    "lj_probe_join_noalloc", "lj_probe_join_noalloc_max_keys",
)
GAP_SLOT = 0xFFFFFFFF  # payload of a gap slot in lj_gapped_slots_host


class LJError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class lj_index_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("leaves", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("nonempty_leaves", ctypes.c_uint32),
        ("max_leaf_keys", ctypes.c_uint32),
        ("max_mult", ctypes.c_uint64),
        ("mean_window", ctypes.c_double),
        ("max_window", ctypes.c_uint64),
        ("device_bytes", ctypes.c_uint64),
        ("root_a0", ctypes.c_double),
        ("root_b0", ctypes.c_double),
        ("root_kmin", ctypes.c_uint64),
        ("slots_per_key", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
        ("nslots", ctypes.c_uint64),
    ]


class lj_batch_desc(ctypes.Structure):
    _fields_ = [
        ("index", ctypes.c_void_p),
        ("s_keys_dev", ctypes.c_void_p),
        ("m", ctypes.c_uint64),
        ("out_pairs_dev", ctypes.c_void_p),
        ("out_capacity", ctypes.c_uint64),
        ("out_count_dev", ctypes.c_void_p),
    ]


class lj_batch_tuning(ctypes.Structure):
    _fields_ = [
        ("keys_per_lane", ctypes.c_uint32 * 4),
        ("branches", ctypes.c_uint32),
        ("use_graph", ctypes.c_uint32),
        ("binned_min_keys", ctypes.c_uint64),
        ("measured_ms", ctypes.c_float),
        ("fused", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {"keys_per_lane": list(self.keys_per_lane), "branches": self.branches,
                "use_graph": self.use_graph, "binned_min_keys": self.binned_min_keys,
                "fused": self.fused, "measured_ms": self.measured_ms}


class lj_server_config(ctypes.Structure):
    _fields_ = [
        ("budget_bytes", ctypes.c_uint64),
        ("slots", ctypes.c_uint32),
        ("max_batch_requests", ctypes.c_uint32),
        ("max_batch_keys", ctypes.c_uint64),
        ("keys_per_lane", ctypes.c_uint32 * 4),
        ("binned_min_keys", ctypes.c_uint64),
        ("fused", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
    ]


class lj_request_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("batch_size", ctypes.c_uint32),
        ("count", ctypes.c_uint64),
        ("submit_ns", ctypes.c_uint64),
        ("start_ns", ctypes.c_uint64),
        ("done_ns", ctypes.c_uint64),
    ]


class lj_replay_request(ctypes.Structure):
    _fields_ = [
        ("index_id", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
        ("s_keys_dev", ctypes.c_void_p),
        ("m", ctypes.c_uint64),
        ("out_pairs_dev", ctypes.c_void_p),
        ("out_capacity", ctypes.c_uint64),
        ("arrival_ns", ctypes.c_uint64),
    ]


class lj_server_stats(ctypes.Structure):
    _fields_ = [
        ("requests_done", ctypes.c_uint64),
        ("batches", ctypes.c_uint64),
        ("peak_bytes_in_use", ctypes.c_uint64),
        ("peak_queue", ctypes.c_uint64),
        ("max_batch_size", ctypes.c_uint64),
        ("keys_probed", ctypes.c_uint64),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblj.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2111_08824_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.lj_build_rmi.argtypes = [vp, u64, u32, u32, vp, ctypes.POINTER(vp)]
        L.lj_build_rmi_host_only.argtypes = [vp, u64, u32, u32, ctypes.POINTER(vp)]
        L.lj_build_gapped_rmi.argtypes = [vp, u64, u32, u32, u32, vp, ctypes.POINTER(vp)]
        L.lj_build_gapped_rmi_host_only.argtypes = [vp, u64, u32, u32, u32, ctypes.POINTER(vp)]
        L.lj_gapped_slots_host.argtypes = [vp, vp, vp, u64, ctypes.POINTER(u64)]
        L.lj_build_learned_hash.argtypes = [vp, u64, u32, u32, u32, vp, ctypes.POINTER(vp)]
        L.lj_build_learned_hash_host_only.argtypes = [vp, u64, u32, u32, u32,
                                                      ctypes.POINTER(vp)]
        L.lj_hash_buckets_host.argtypes = [vp, vp, vp, vp, u64, ctypes.POINTER(u64),
                                           ctypes.POINTER(u64)]
        L.lj_free_index.argtypes = [vp]
        L.lj_free_index.restype = None
        L.lj_probe_join.argtypes = [vp, vp, u64, vp, u64, ctypes.POINTER(u64), vp]
        L.lj_probe_workspace_bytes.argtypes = [vp, u64]
        L.lj_probe_workspace_bytes.restype = u64
        L.lj_probe_join_async.argtypes = [vp, vp, u64, vp, u64, vp, vp, u64, vp]
        L.lj_index_get_stats.argtypes = [vp, ctypes.POINTER(lj_index_stats)]
        L.lj_self_check.argtypes = [vp, ctypes.POINTER(u64), vp]
        L.lj_predict_windows.argtypes = [vp, vp, u64, vp, vp, vp, vp, vp]
        L.lj_predict_windows_host.argtypes = [vp, vp, u64, vp, vp, vp, vp]
        L.lj_probe_set_timing_events.argtypes = [vp, vp]
        L.lj_bench_random_gather.argtypes = [vp, u64, u32, u64, u64, vp, vp]
        L.lj_batch_default_tuning.argtypes = [ctypes.POINTER(lj_batch_tuning)]
        L.lj_batch_default_tuning.restype = None
        L.lj_batch_plan_create.argtypes = [ctypes.POINTER(lj_batch_desc), u32,
                                           ctypes.POINTER(lj_batch_tuning), ctypes.POINTER(vp)]
        L.lj_batch_plan_run.argtypes = [vp, vp]
        L.lj_batch_plan_destroy.argtypes = [vp]
        L.lj_batch_plan_destroy.restype = None
        L.lj_batch_autotune.argtypes = [ctypes.POINTER(lj_batch_desc), u32, vp,
                                        ctypes.POINTER(lj_batch_tuning)]
        L.lj_server_default_config.argtypes = [ctypes.POINTER(lj_server_config), u64]
        L.lj_server_default_config.restype = None
        L.lj_server_create.argtypes = [ctypes.POINTER(vp), u32, ctypes.POINTER(lj_server_config),
                                       ctypes.POINTER(vp)]
        L.lj_server_submit.argtypes = [vp, u32, vp, u64, vp, u64, ctypes.POINTER(u64)]
        L.lj_server_submit_device.argtypes = [vp, u32, vp, u64, vp, u64, ctypes.POINTER(u64)]
        L.lj_server_wait.argtypes = [vp, u64, ctypes.c_int64, ctypes.POINTER(lj_request_result)]
        L.lj_server_replay.argtypes = [vp, ctypes.POINTER(lj_replay_request), u64,
                                       ctypes.POINTER(lj_request_result)]
        L.lj_server_get_stats.argtypes = [vp, ctypes.POINTER(lj_server_stats)]
        L.lj_server_destroy.argtypes = [vp]
        L.lj_server_destroy.restype = None
        L.lj_sort_join_workspace_bytes.argtypes = [u64, u64]
        L.lj_sort_join_workspace_bytes.restype = u64
        L.lj_sort_join_async.argtypes = [vp, u64, vp, u64, vp, u64, vp, vp, u64, vp]
        L.lj_learned_sort_async.argtypes = [vp, u64, vp, vp, vp, u64, vp]
        L.lj_probe_join_noalloc.argtypes = [vp, vp, u64, vp, u64, vp, vp]
        L.lj_probe_join_noalloc_max_keys.argtypes = []
        L.lj_probe_join_noalloc_max_keys.restype = u64
        L.lj_strerror.argtypes = [i32]
        L.lj_strerror.restype = ctypes.c_char_p
        for f in ("lj_build_rmi", "lj_build_rmi_host_only", "lj_probe_join",
                  "lj_probe_join_async", "lj_index_get_stats", "lj_self_check",
                  "lj_predict_windows", "lj_predict_windows_host",
                  "lj_probe_set_timing_events", "lj_bench_random_gather",
                  "lj_batch_plan_create", "lj_batch_plan_run", "lj_batch_autotune",
                  "lj_server_create", "lj_server_submit", "lj_server_submit_device",
                  "lj_server_wait", "lj_server_replay",
                  "lj_server_get_stats", "lj_sort_join_async", "lj_learned_sort_async",
                  "lj_probe_join_noalloc"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().lj_strerror(int(status)).decode()


def _check(status: int, what: str) -> int:
    if status != LJ_OK:
        raise LJError(status, what)
    return status


def _stream_ptr(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t) -> int:
    if t is None:
        return 0
    assert t.is_cuda and t.is_contiguous()
    return t.data_ptr()


def _host_u64(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint64:
        a = a.astype(np.uint64)
    return a


class Index:
    """Owner of an lj_index handle."""

    def __init__(self, handle: int, host_only: bool):
        self.handle = handle
        self.host_only = host_only

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lj_free_index(self.handle)
        self.handle = None

    @property
    def stats(self) -> lj_index_stats:
        st = lj_index_stats()
        _check(lib().lj_index_get_stats(self.handle, ctypes.byref(st)), "lj_index_get_stats")
        return st


def lj_build_rmi(r_keys, leaves: int, flags: int = LJ_LEAF_FP32, stream=None) -> Index:
    """Build the index over host array r_keys (sorted uint64)."""
    R = _host_u64(r_keys)
    h = ctypes.c_void_p()
    _check(lib().lj_build_rmi(R.ctypes.data if len(R) else None, len(R), leaves, flags,
                              _stream_ptr(stream), ctypes.byref(h)), "lj_build_rmi")
    return Index(h.value, False)


def lj_build_rmi_host_only(r_keys, leaves: int, flags: int = LJ_LEAF_FP32) -> Index:
    R = _host_u64(r_keys)
    h = ctypes.c_void_p()
    _check(lib().lj_build_rmi_host_only(R.ctypes.data if len(R) else None, len(R), leaves,
                                        flags, ctypes.byref(h)), "lj_build_rmi_host_only")
    return Index(h.value, True)


def lj_build_gapped_rmi(r_keys, leaves: int, slots_per_key: int = 4, flags: int = LJ_LEAF_FP32,
                        stream=None) -> Index:
    """Build a gapped RMI over host array r_keys (sorted uint64)."""
    R = _host_u64(r_keys)
    h = ctypes.c_void_p()
    _check(lib().lj_build_gapped_rmi(R.ctypes.data if len(R) else None, len(R), leaves,
                                     slots_per_key, flags, _stream_ptr(stream), ctypes.byref(h)),
           "lj_build_gapped_rmi")
    return Index(h.value, False)


def lj_build_gapped_rmi_host_only(r_keys, leaves: int, slots_per_key: int = 4,
                                  flags: int = LJ_LEAF_FP32) -> Index:
    R = _host_u64(r_keys)
    h = ctypes.c_void_p()
    _check(lib().lj_build_gapped_rmi_host_only(R.ctypes.data if len(R) else None, len(R),
                                               leaves, slots_per_key, flags, ctypes.byref(h)),
           "lj_build_gapped_rmi_host_only")
    return Index(h.value, True)


def lj_gapped_slots_host(index: Index):
    """(keys uint64[nslots], ridx uint32[nslots]) of a host-only gapped index;
    a gap has ridx == GAP_SLOT and holds the next key of R."""
    n = ctypes.c_uint64()
    st = lib().lj_gapped_slots_host(index.handle, None, None, 0, ctypes.byref(n))
    if st not in (LJ_OK, LJ_ERR_CAPACITY):
        _check(st, "lj_gapped_slots_host")
    keys = np.empty(n.value, dtype=np.uint64)
    ridx = np.empty(n.value, dtype=np.uint32)
    _check(lib().lj_gapped_slots_host(index.handle, keys.ctypes.data, ridx.ctypes.data, n.value,
                                      ctypes.byref(n)), "lj_gapped_slots_host")
    return keys, ridx


def lj_build_learned_hash(r_keys, leaves: int, slots_per_key: int = 4,
                          flags: int = LJ_LEAF_FP32, stream=None) -> Index:
    """Build a learned hash index over host array r_keys (sorted uint64)."""
    R = _host_u64(r_keys)
    h = ctypes.c_void_p()
    _check(lib().lj_build_learned_hash(R.ctypes.data if len(R) else None, len(R), leaves,
                                       slots_per_key, flags, _stream_ptr(stream),
                                       ctypes.byref(h)), "lj_build_learned_hash")
    return Index(h.value, False)


def lj_build_learned_hash_host_only(r_keys, leaves: int, slots_per_key: int = 4,
                                    flags: int = LJ_LEAF_FP32) -> Index:
    R = _host_u64(r_keys)
    h = ctypes.c_void_p()
    _check(lib().lj_build_learned_hash_host_only(R.ctypes.data if len(R) else None, len(R),
                                                 leaves, slots_per_key, flags, ctypes.byref(h)),
           "lj_build_learned_hash_host_only")
    return Index(h.value, True)


def lj_hash_buckets_host(index: Index):
    """(keys uint64[nb, 4], ridx uint32[nb, 4], next uint32[nb], nprimary) of
    a host-only learned hash index; an empty slot has ridx == GAP_SLOT, the
    end of a chain next == GAP_SLOT."""
    n = ctypes.c_uint64()
    npri = ctypes.c_uint64()
    st = lib().lj_hash_buckets_host(index.handle, None, None, None, 0, ctypes.byref(n),
                                    ctypes.byref(npri))
    if st not in (LJ_OK, LJ_ERR_CAPACITY):
        _check(st, "lj_hash_buckets_host")
    keys = np.empty((n.value, 4), dtype=np.uint64)
    ridx = np.empty((n.value, 4), dtype=np.uint32)
    nxt = np.empty(n.value, dtype=np.uint32)
    _check(lib().lj_hash_buckets_host(index.handle, keys.ctypes.data, ridx.ctypes.data,
                                      nxt.ctypes.data, n.value, ctypes.byref(n),
                                      ctypes.byref(npri)), "lj_hash_buckets_host")
    return keys, ridx, nxt, npri.value


def lj_probe_join(index: Index, s_keys_dev, out_pairs_dev=None, stream=None):
    """Probe with device tensor s_keys_dev (int64 storage of uint64 keys).

    out_pairs_dev: int32 tensor of shape (cap, 2) or None (count only).
    Returns (status, count); status is LJ_OK or LJ_ERR_CAPACITY.
    """
    m = s_keys_dev.numel()
    cap = 0 if out_pairs_dev is None else out_pairs_dev.shape[0]
    cnt = ctypes.c_uint64()
    st = lib().lj_probe_join(index.handle, _dev_ptr(s_keys_dev) if m else None, m,
                             _dev_ptr(out_pairs_dev) if cap else None, cap,
                             ctypes.byref(cnt), _stream_ptr(stream))
    if st not in (LJ_OK, LJ_ERR_CAPACITY):
        raise LJError(st, "lj_probe_join")
    return st, cnt.value


def lj_probe_workspace_bytes(index: Index, m: int) -> int:
    return int(lib().lj_probe_workspace_bytes(index.handle, m))


def lj_probe_join_async(index: Index, s_keys_dev, out_pairs_dev, count_dev, workspace_dev,
                        stream=None) -> None:
    """Enqueue a probe; count_dev is a device int64 tensor of one element."""
    m = s_keys_dev.numel()
    cap = 0 if out_pairs_dev is None else out_pairs_dev.shape[0]
    ws_bytes = 0 if workspace_dev is None else workspace_dev.numel() * workspace_dev.element_size()
    _check(lib().lj_probe_join_async(index.handle, _dev_ptr(s_keys_dev) if m else None, m,
                                     _dev_ptr(out_pairs_dev) if cap else None, cap,
                                     _dev_ptr(count_dev), _dev_ptr(workspace_dev), ws_bytes,
                                     _stream_ptr(stream)), "lj_probe_join_async")


def lj_probe_join_noalloc(index: Index, s_keys_dev, out_pairs_dev, count_dev,
                          stream=None) -> None:
    """Enqueue a direct probe whose workspace is the library's fixed device
    array (nothing is allocated); count_dev is a device int64 tensor of one
    element.  Calls on one GPU must not overlap."""
    m = s_keys_dev.numel()
    cap = 0 if out_pairs_dev is None else out_pairs_dev.shape[0]
    _check(lib().lj_probe_join_noalloc(index.handle, _dev_ptr(s_keys_dev) if m else None, m,
                                       _dev_ptr(out_pairs_dev) if cap else None, cap,
                                       _dev_ptr(count_dev), _stream_ptr(stream)),
           "lj_probe_join_noalloc")


def lj_probe_join_noalloc_max_keys() -> int:
    return int(lib().lj_probe_join_noalloc_max_keys())


def lj_sort_join_workspace_bytes(n: int, m: int) -> int:
    return int(lib().lj_sort_join_workspace_bytes(n, m))


def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


def lj_sort_join_async(r_keys_dev, s_keys_dev, out_pairs_dev, count_dev, workspace_dev,
                       stream=None) -> None:
    """Enqueue a learned sort join of two device key tensors in any order;
    count_dev is a device int64 tensor of one element."""
    n, m = r_keys_dev.numel(), s_keys_dev.numel()
    cap = 0 if out_pairs_dev is None else out_pairs_dev.shape[0]
    _check(lib().lj_sort_join_async(_dev_ptr(r_keys_dev) if n else None, n,
                                    _dev_ptr(s_keys_dev) if m else None, m,
                                    _dev_ptr(out_pairs_dev) if cap else None, cap,
                                    _dev_ptr(count_dev), _dev_ptr(workspace_dev),
                                    _nbytes(workspace_dev), _stream_ptr(stream)),
           "lj_sort_join_async")


def lj_learned_sort_async(keys_dev, sorted_keys_dev, positions_dev, workspace_dev,
                          stream=None) -> None:
    """Enqueue the learned sort of a device key tensor into (key, position)
    order: sorted keys (int64/uint64 view) and int32 input positions."""
    n = keys_dev.numel()
    _check(lib().lj_learned_sort_async(_dev_ptr(keys_dev) if n else None, n,
                                       _dev_ptr(sorted_keys_dev) if n else None,
                                       _dev_ptr(positions_dev) if n else None,
                                       _dev_ptr(workspace_dev), _nbytes(workspace_dev),
                                       _stream_ptr(stream)), "lj_learned_sort_async")


def lj_self_check(index: Index, stream=None) -> int:
    v = ctypes.c_uint64()
    _check(lib().lj_self_check(index.handle, ctypes.byref(v), _stream_ptr(stream)),
           "lj_self_check")
    return v.value


def lj_predict_windows(index: Index, keys_dev, leaf_dev, pred_dev, lo_dev, hi_dev,
                       stream=None) -> None:
    _check(lib().lj_predict_windows(index.handle, _dev_ptr(keys_dev), keys_dev.numel(),
                                    _dev_ptr(leaf_dev), _dev_ptr(pred_dev), _dev_ptr(lo_dev),
                                    _dev_ptr(hi_dev), _stream_ptr(stream)),
           "lj_predict_windows")


def lj_predict_windows_host(index: Index, keys):
    """(leaf, pred, lo, hi) arrays for host keys."""
    keys = _host_u64(keys)
    m = len(keys)
    leaf = np.empty(m, dtype=np.uint32)
    pred = np.empty(m, dtype=np.int64)
    lo = np.empty(m, dtype=np.int64)
    hi = np.empty(m, dtype=np.int64)
    _check(lib().lj_predict_windows_host(index.handle, keys.ctypes.data if m else None, m,
                                         leaf.ctypes.data, pred.ctypes.data, lo.ctypes.data,
                                         hi.ctypes.data), "lj_predict_windows_host")
    return leaf, pred, lo, hi


def lj_probe_set_timing_events(start, stop) -> None:
    """start/stop: torch.cuda.Event objects (or None to disable)."""
    _check(lib().lj_probe_set_timing_events(
        start.cuda_event if start is not None else None,
        stop.cuda_event if stop is not None else None), "lj_probe_set_timing_events")


def lj_bench_random_gather(buf_dev, granule: int, reads: int, seed: int, sink_dev,
                           stream=None) -> None:
    nbytes = buf_dev.numel() * buf_dev.element_size()
    _check(lib().lj_bench_random_gather(_dev_ptr(buf_dev), nbytes, granule, reads, seed,
                                        _dev_ptr(sink_dev), _stream_ptr(stream)),
           "lj_bench_random_gather")


def make_batch_descs(batches):
    """batches: list of (Index, s_keys_dev, out_pairs_dev or None, count_dev)."""
    arr = (lj_batch_desc * len(batches))()
    for i, (ix, s, out, cnt) in enumerate(batches):
        arr[i].index = ix.handle
        arr[i].s_keys_dev = _dev_ptr(s) if s.numel() else None
        arr[i].m = s.numel()
        arr[i].out_pairs_dev = _dev_ptr(out) if out is not None and out.shape[0] else None
        arr[i].out_capacity = 0 if out is None else out.shape[0]
        arr[i].out_count_dev = _dev_ptr(cnt)
    return arr


def lj_batch_default_tuning() -> lj_batch_tuning:
    t = lj_batch_tuning()
    lib().lj_batch_default_tuning(ctypes.byref(t))
    return t


class BatchPlan:
    """Owner of an lj_batch_plan handle (keeps its descriptor inputs alive)."""

    def __init__(self, batches, tuning: lj_batch_tuning | None = None):
        self._batches = batches
        descs = make_batch_descs(batches)
        h = ctypes.c_void_p()
        _check(lib().lj_batch_plan_create(descs, len(batches),
                                          ctypes.byref(tuning) if tuning is not None else None,
                                          ctypes.byref(h)), "lj_batch_plan_create")
        self.handle = h.value

    def run(self, stream=None) -> None:
        _check(lib().lj_batch_plan_run(self.handle, _stream_ptr(stream)), "lj_batch_plan_run")

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lj_batch_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


def lj_batch_autotune(batches, stream=None) -> lj_batch_tuning:
    t = lj_batch_tuning()
    _check(lib().lj_batch_autotune(make_batch_descs(batches), len(batches),
                                   _stream_ptr(stream), ctypes.byref(t)), "lj_batch_autotune")
    return t


def lj_server_default_config(budget_bytes: int) -> lj_server_config:
    c = lj_server_config()
    lib().lj_server_default_config(ctypes.byref(c), budget_bytes)
    return c


class Server:
    """Owner of an lj_server handle.  Host buffers passed to submit() must
    stay alive until wait() returns for that ticket (numpy arrays, ideally
    backed by pinned memory)."""

    def __init__(self, indexes, config: lj_server_config):
        self._indexes = list(indexes)
        arr = (ctypes.c_void_p * len(indexes))(*[ix.handle for ix in indexes])
        h = ctypes.c_void_p()
        _check(lib().lj_server_create(arr, len(indexes), ctypes.byref(config), ctypes.byref(h)),
               "lj_server_create")
        self.handle = h.value

    def submit(self, index_id: int, s_keys_host: np.ndarray, out_pairs_host) -> int:
        """out_pairs_host: uint32 array of shape (cap, 2), or None."""
        assert s_keys_host.dtype == np.uint64 and s_keys_host.flags["C_CONTIGUOUS"]
        cap = 0 if out_pairs_host is None else out_pairs_host.shape[0]
        t = ctypes.c_uint64()
        _check(lib().lj_server_submit(self.handle, index_id,
                                      s_keys_host.ctypes.data if len(s_keys_host) else None,
                                      len(s_keys_host),
                                      out_pairs_host.ctypes.data if cap else None, cap,
                                      ctypes.byref(t)), "lj_server_submit")
        return t.value

    def submit_device(self, index_id: int, s_keys_dev, out_pairs_dev) -> int:
        """Device-resident request: s_keys_dev an int64 CUDA tensor of keys,
        out_pairs_dev an (cap, 2) int32 CUDA tensor or None; the work that
        writes them must be complete (the server's streams do not wait for
        torch's), and both must stay alive and untouched until wait()
        returns for the ticket."""
        m = s_keys_dev.numel()
        cap = 0 if out_pairs_dev is None else out_pairs_dev.shape[0]
        t = ctypes.c_uint64()
        _check(lib().lj_server_submit_device(self.handle, index_id,
                                             _dev_ptr(s_keys_dev) if m else None, m,
                                             _dev_ptr(out_pairs_dev) if cap else None, cap,
                                             ctypes.byref(t)), "lj_server_submit_device")
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> lj_request_result:
        r = lj_request_result()
        _check(lib().lj_server_wait(self.handle, ticket, timeout_ms, ctypes.byref(r)),
               "lj_server_wait")
        return r

    def replay(self, requests, arrival_ns=None):
        """Submit device-resident requests from a native thread at their
        arrival times (ns after the start; None = all at once) and wait for
        them all.  requests: list of (index_id, s_keys_dev, out_pairs_dev or
        None).  Returns the list of lj_request_result."""
        n = len(requests)
        arr = (lj_replay_request * n)()
        for i, (ix, s, out) in enumerate(requests):
            r = arr[i]
            r.index_id = ix
            r.m = s.numel()
            r.s_keys_dev = _dev_ptr(s) if r.m else None
            r.out_capacity = 0 if out is None else out.shape[0]
            r.out_pairs_dev = _dev_ptr(out) if r.out_capacity else None
            r.arrival_ns = 0 if arrival_ns is None else int(arrival_ns[i])
        res = (lj_request_result * n)()
        _check(lib().lj_server_replay(self.handle, arr, n, res), "lj_server_replay")
        return list(res)

    @property
    def stats(self) -> lj_server_stats:
        s = lj_server_stats()
        _check(lib().lj_server_get_stats(self.handle, ctypes.byref(s)), "lj_server_get_stats")
        return s

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lj_server_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# Convenience wrappers used by tests and the benchmark.

def to_device_keys(a: np.ndarray, device="cuda"):
    """uint64 numpy array -> int64 CUDA tensor with the same bits."""
    import torch
    a = _host_u64(a)
    return torch.from_numpy(a.view(np.int64)).to(device)


def probe(index: Index, s_keys_dev, capacity: int | None = None, stream=None):
    """Probe and return the pairs as an (count, 2) int32 CUDA tensor.

    With capacity None, a count-only probe sizes the output first."""
    import torch
    if capacity is None:
        _, capacity = lj_probe_join(index, s_keys_dev, None, stream)
    out = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=s_keys_dev.device)
    st, cnt = lj_probe_join(index, s_keys_dev, out[:capacity] if capacity else None, stream)
    if st == LJ_ERR_CAPACITY:
        out = torch.empty((cnt, 2), dtype=torch.int32, device=s_keys_dev.device)
        st, cnt = lj_probe_join(index, s_keys_dev, out, stream)
        _check(st, "lj_probe_join")
    return out[:cnt]


def sort_join(r_keys_dev, s_keys_dev, capacity: int | None = None, stream=None):
    """Learned sort join of two device key tensors in any order; returns the
    (count, 2) int32 CUDA tensor of (s_idx, r_idx) pairs and the true count.

    With capacity None, a count-only join sizes the output first."""
    import torch
    dev = s_keys_dev.device
    n, m = r_keys_dev.numel(), s_keys_dev.numel()
    ws = torch.empty(max(lj_sort_join_workspace_bytes(n, m), 1), dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    if capacity is None:
        lj_sort_join_async(r_keys_dev, s_keys_dev, None, cnt, ws, stream)
        torch.cuda.synchronize(dev)
        capacity = int(cnt.item())
    out = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=dev)
    lj_sort_join_async(r_keys_dev, s_keys_dev, out if capacity else None, cnt, ws, stream)
    torch.cuda.synchronize(dev)
    count = int(cnt.item())
    return out[:min(count, capacity)], count


def learned_sort(keys_dev, stream=None):
    """(sorted keys as int64 bits, int32 input positions) of a device key tensor."""
    import torch
    dev = keys_dev.device
    n = keys_dev.numel()
    ws = torch.empty(max(lj_sort_join_workspace_bytes(n, 0), 1), dtype=torch.uint8, device=dev)
    ko = torch.empty(n, dtype=torch.int64, device=dev)
    po = torch.empty(n, dtype=torch.int32, device=dev)
    lj_learned_sort_async(keys_dev, ko, po, ws, stream)
    torch.cuda.synchronize(dev)
    return ko, po
