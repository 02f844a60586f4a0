"""GPU parity of the batched probe (many indexes in one plan: fused probe
kernels forked over parallel streams, replayed from a HIP graph) against the
oracle, batch by batch."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2111_08824_amd import lj

pytestmark = pytest.mark.gpu


def _mixed_batches(seed=7):
    """Indexes of every kind (FP32/FP64 leaves, unique/duplicate keys) and
    batch sizes from empty to several tiles of every size class."""
    import torch
    ws = workloads.multi_index_batches(k=10, seed=seed, n_lo=1e3, n_hi=3e5, m_lo=1, m_hi=3e5)
    dup = workloads.c3_dup_runs(seed=seed, scale=0.002)
    ws.append(dup)
    items = []
    for i, w in enumerate(ws):
        flags = lj.LJ_LEAF_FP64 if i % 3 == 1 else lj.LJ_LEAF_FP32
        if i % 4 == 2:
            flags |= lj.LJ_ROOT_RADIX
        S = w.S if i != 4 else w.S[:0]  # one empty batch
        ix = lj.lj_build_rmi(w.R, w.leaves, flags)
        cap = max(1, len(S) * int(ix.stats.max_mult))
        s = lj.to_device_keys(S)
        out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        items.append((w.R, S, ix, s, out, cnt))
    return items


def _check(items):
    for R, S, ix, s, out, cnt in items:
        want = oracle.sort_merge_join(R, S)
        got_n = int(cnt.item())
        assert got_n == len(want), (len(R), len(S), got_n, len(want))
        got = out[:got_n].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("binned_min_keys", [0, 1, 5000])
def test_plan_matches_oracle_on_every_replay(use_graph, binned_min_keys, fused):
    import torch
    items = _mixed_batches()
    t = lj.lj_batch_default_tuning()
    t.use_graph = use_graph
    t.fused = fused  # one kernel for the direct batches of each kernel group, or one per batch
    t.binned_min_keys = binned_min_keys  # index flags / every batch binned / large ones
    plan = lj.BatchPlan([(ix, s, out, cnt) for _, _, ix, s, out, cnt in items], t)
    for rep in range(3):
        print(f"[batches] replay {rep} graph={use_graph} binned_min_keys={binned_min_keys} "
              f"fused={fused}", flush=True)
        for *_, out, cnt in items:  # eager work between replays
            out.fill_(-1)
            cnt.fill_(-7)
        plan.run()
        torch.cuda.synchronize()
        _check(items)
    plan.close()


def test_plan_sees_new_key_values():
    import torch
    items = _mixed_batches(seed=8)
    plan = lj.BatchPlan([(ix, s, out, cnt) for _, _, ix, s, out, cnt in items])
    plan.run()
    torch.cuda.synchronize()
    _check(items)
    # overwrite the outer keys in place and replay the same graph
    new_items = []
    for j, (R, S, ix, s, out, cnt) in enumerate(items):
        if len(S):
            S2 = workloads.gen.probe_mix(R, len(S), 0.3, 100 + j, miss_hi=int(R[-1]) + 10)
            s.copy_(lj.to_device_keys(S2))
            S = S2
        new_items.append((R, S, ix, s, out, cnt))
    plan.run()
    torch.cuda.synchronize()
    _check(new_items)


def test_capacity_in_a_batch():
    import torch
    w = workloads.c3_dup_runs(scale=0.001)
    want = oracle.sort_merge_join(w.R, w.S)
    ix = lj.lj_build_rmi(w.R, w.leaves)
    s = lj.to_device_keys(w.S)
    cap = len(want) // 2
    out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    cnt2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan = lj.BatchPlan([(ix, s, out, cnt), (ix, s, None, cnt2)])
    plan.run()
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want) and int(cnt2.item()) == len(want)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want[:cap])


def test_autotune_then_plan():
    import torch
    items = _mixed_batches(seed=9)
    batches = [(ix, s, out, cnt) for _, _, ix, s, out, cnt in items]
    t = lj.lj_batch_autotune(batches)
    print("[batches] tuned", t.as_dict(), flush=True)
    assert t.measured_ms > 0
    assert all(k in (4, 8, 16, 24) for k in t.keys_per_lane)
    assert 1 <= t.branches <= 16
    plan = lj.BatchPlan(batches, t)
    for *_, out, cnt in items:
        out.fill_(-1)
        cnt.fill_(-7)
    plan.run()
    torch.cuda.synchronize()
    _check(items)


@pytest.mark.parametrize("kpl", [4, 8, 16, 24])
def test_fused_plan_tile_shapes_and_many_batches(kpl):
    # Many small and ragged batches of every kernel group (FP32 / FP64
    # leaves, unique / duplicate keys, linear and radix roots, plain and
    # gapped RMIs) in one fused plan; each size class with the given keys
    # per lane (16 and 24 run as 8).
    import torch
    rng = np.random.default_rng(kpl)
    items = []
    for i in range(40):
        n = int(rng.integers(1, 60_000))
        if i % 5 == 4:
            R = np.repeat(workloads.gen.uniform_unique(max(1, n // 4), 30, i), 4)
        else:
            R = workloads.gen.uniform_unique(n, 30, i)
        m = int(rng.choice([1, 255, 1023, 1024, 1025, 4097, 20_000, 70_001]))
        S = workloads.gen.probe_mix(R, m, 0.5, 1000 + i, miss_hi=2**30)
        flags = (lj.LJ_LEAF_FP64 if i % 3 == 0 else lj.LJ_LEAF_FP32) | \
            (lj.LJ_ROOT_RADIX if i % 2 else 0)
        if i % 7 in (3, 4):  # gapped RMIs (both leaf kinds, unique and duplicate keys)
            ix = lj.lj_build_gapped_rmi(R, max(1, n // 200), 1 + i % 5, flags)
        else:
            ix = lj.lj_build_rmi(R, max(1, n // 200), flags)
        cap = max(1, m * int(ix.stats.max_mult))
        s = lj.to_device_keys(S)
        out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        items.append((R, S, ix, s, out, cnt))
    t = lj.lj_batch_default_tuning()
    t.keys_per_lane[:] = [kpl] * 4
    t.fused = 1
    plan = lj.BatchPlan([(ix, s, out, cnt) for _, _, ix, s, out, cnt in items], t)
    for rep in range(2):
        print(f"[batches] fused kpl={kpl} replay {rep}", flush=True)
        for *_, out, cnt in items:
            out.fill_(-1)
            cnt.fill_(-7)
        plan.run()
        torch.cuda.synchronize()
        _check(items)
    plan.close()


def test_plan_argument_errors():
    import torch
    w = workloads.c1_uniform(scale=0.01)
    ix = lj.lj_build_rmi(w.R, w.leaves)
    s = lj.to_device_keys(w.S)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    host = lj.lj_build_rmi_host_only(w.R, w.leaves)
    with pytest.raises(lj.LJError) as e:
        lj.BatchPlan([(host, s, None, cnt)])
    assert e.value.status == lj.LJ_ERR_ARG
    t = lj.lj_batch_default_tuning()
    t.keys_per_lane[2] = 12
    with pytest.raises(lj.LJError) as e:
        lj.BatchPlan([(ix, s, None, cnt)], t)
    assert e.value.status == lj.LJ_ERR_ARG
