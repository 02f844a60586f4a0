"""The probe entry point that allocates nothing (its workspace is the
library's fixed device array) gives exactly the pairs and count of
lj_probe_join_async with a caller workspace, on two calls in a row on one
stream, the second with a smaller input (the array keeps the first call's
contents and must be cleared by the call itself)."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from paper_2111_08824_amd import lj

pytestmark = pytest.mark.gpu


def _async_reference(ix, s, cap):
    import torch
    out = torch.full((max(cap, 1), 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(256, lj.lj_probe_workspace_bytes(ix, s.numel())), dtype=torch.uint8,
                     device="cuda")
    lj.lj_probe_join_async(ix, s, out if cap else None, cnt, ws)
    torch.cuda.synchronize()
    return out, int(cnt.item())


def test_noalloc_equals_async_on_two_calls_in_a_row():
    import torch
    big = workloads.c3_dup_runs(scale=0.004)           # 4e5 rows, duplicates
    small = workloads.c2_lognormal_zipf(scale=0.0004)  # 8e4 keys, unique
    cases = []
    for w, flags in ((big, lj.LJ_LEAF_FP32 | lj.LJ_PROBE_BINNED), (small, lj.LJ_LEAF_FP64)):
        ix = lj.lj_build_rmi(w.R, w.leaves, flags)
        s = lj.to_device_keys(w.S)
        want = oracle.sort_merge_join(w.R, w.S)
        cases.append((w, ix, s, want))
    assert len(cases[1][0].S) < len(cases[0][0].S)
    stream = torch.cuda.current_stream()
    results = []
    for w, ix, s, want in cases:  # back to back on one stream, no sync between
        cap = len(want)
        out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        lj.lj_probe_join_noalloc(ix, s, out, cnt, stream)
        results.append((out, cnt))
    torch.cuda.synchronize()
    for (w, ix, s, want), (out, cnt) in zip(cases, results):
        print(f"[noalloc] {w.name}: m={len(w.S)} pairs={len(want)}", flush=True)
        ref_out, ref_cnt = _async_reference(ix, s, len(want))
        assert int(cnt.item()) == ref_cnt == len(want)
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref_out[:ref_cnt].cpu().numpy().view(np.uint32))
        assert np.array_equal(got, want)


def test_noalloc_capacity_count_only_and_limits():
    import torch
    w = workloads.c1_uniform(scale=0.05)
    ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32)
    s = lj.to_device_keys(w.S)
    want = oracle.sort_merge_join(w.R, w.S)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    lj.lj_probe_join_noalloc(ix, s, None, cnt)  # count only
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    cap = len(want) // 3
    out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    lj.lj_probe_join_noalloc(ix, s, out, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want[:cap])
    lj.lj_probe_join_noalloc(ix, s[:0], None, cnt)  # no keys
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    # Sizes beyond the fixed array are refused before any device work.
    too_many = lj.lj_probe_join_noalloc_max_keys() + 1
    st = lj.lib().lj_probe_join_noalloc(ix.handle, s.data_ptr(), too_many, None, 0,
                                        cnt.data_ptr(), ctypes.c_void_p(0))
    assert st == lj.LJ_ERR_TOO_LARGE
