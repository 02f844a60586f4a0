"""GPU tests of the serving loop: each request's result is the same alone
and in the mix (exact: join output is integer work), admission respects the
memory budget, batches form under load, oversize requests are rejected."""
import threading
import time

import numpy as np
import pytest

import oracle
import workloads
from paper_2111_08824_amd import lj

pytestmark = pytest.mark.gpu


def _indexes():
    ws = [workloads.c1_uniform(scale=0.2), workloads.c3_dup_runs(scale=0.002),
          workloads.c2_lognormal_zipf(scale=0.001), workloads.c2_lognormal_zipf(scale=0.002)]
    ixs = [lj.lj_build_rmi(w.R, w.leaves, (lj.LJ_LEAF_FP32 if i != 1 else lj.LJ_LEAF_FP64)
                           | (lj.LJ_ROOT_RADIX if i == 2 else 0))
           for i, w in enumerate(ws[:3])]
    ixs.append(lj.lj_build_gapped_rmi(ws[3].R, ws[3].leaves, 4,
                                      lj.LJ_LEAF_FP32 | lj.LJ_ROOT_RADIX))
    return ws, ixs


def _requests(ws, n, seed, max_m=200_000):
    rng = np.random.default_rng(seed)
    reqs = []
    for q in range(n):
        i = int(rng.integers(0, len(ws)))
        w = ws[i]
        m = int(np.exp(rng.uniform(0.0, np.log(max_m))))
        if i == 1:  # duplicate-heavy index: about 8.5 pairs per hit
            m = max(1, m // 8)
        a = int(rng.integers(0, max(1, len(w.S) - m)))
        S = np.ascontiguousarray(w.S[a:a + m])
        want = oracle.sort_merge_join(w.R, S)
        cap = len(want) if q % 9 else max(0, len(want) - 5)  # some truncated outputs
        out = np.full((max(cap, 1), 2), 0xFFFFFFFF, dtype=np.uint32)
        reqs.append((i, S, want, cap, out))
    return reqs


def _alone(ix, S):
    return lj.probe(ix, lj.to_device_keys(S)).cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("budget,slots", [(1 << 23, 3), (1 << 30, 4)])
def test_results_alone_equal_results_in_the_mix(budget, slots, fused):
    ws, ixs = _indexes()
    reqs = _requests(ws, 80, seed=budget % 97)
    cfg = lj.lj_server_default_config(budget)
    cfg.slots = slots
    cfg.fused = fused
    srv = lj.Server(ixs, cfg)
    tickets = [None] * len(reqs)
    rng = np.random.default_rng(5)

    def submitter():
        for q, (i, S, want, cap, out) in enumerate(reqs):
            tickets[q] = srv.submit(i, S, out if cap else None)
            if q % 10 == 0:
                time.sleep(0.002 * rng.random())

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    for q, (i, S, want, cap, out) in enumerate(reqs):
        r = srv.wait(tickets[q], 60_000)
        assert r.count == len(want), (q, r.count, len(want))
        if cap >= len(want):
            assert r.status == lj.LJ_OK
        else:
            assert r.status == lj.LJ_ERR_CAPACITY
        got = out[:min(cap, len(want))]
        assert np.array_equal(got, want[:cap])
        alone = _alone(ixs[i], S)
        assert np.array_equal(alone, want)
        assert r.done_ns >= r.start_ns >= r.submit_ns
    st = srv.stats
    print(f"[server] budget={budget} batches={st.batches} max_batch={st.max_batch_size} "
          f"peak_bytes={st.peak_bytes_in_use} peak_queue={st.peak_queue}", flush=True)
    assert st.requests_done == len(reqs)
    assert st.peak_bytes_in_use <= budget
    srv.close()


def test_small_budget_queues_and_batches():
    ws, ixs = _indexes()
    reqs = _requests(ws, 60, seed=11, max_m=20_000)
    cfg = lj.lj_server_default_config(1 << 21)
    cfg.slots = 2
    srv = lj.Server(ixs, cfg)
    tickets = [srv.submit(i, S, out if cap else None) for i, S, want, cap, out in reqs]
    for t, (i, S, want, cap, out) in zip(tickets, reqs):
        r = srv.wait(t, 60_000)
        assert r.count == len(want)
    st = srv.stats
    assert st.peak_queue > 1          # requests waited for admission
    assert st.max_batch_size > 1      # and were batched together
    assert st.peak_bytes_in_use <= (1 << 21)
    srv.close()


def test_oversize_request_and_bad_arguments():
    ws, ixs = _indexes()
    cfg = lj.lj_server_default_config(1 << 16)
    srv = lj.Server(ixs, cfg)
    S = np.ascontiguousarray(ws[0].S[:100_000])
    out = np.empty((100_000, 2), dtype=np.uint32)
    with pytest.raises(lj.LJError) as e:
        srv.submit(0, S, out)
    assert e.value.status == lj.LJ_ERR_TOO_LARGE
    with pytest.raises(lj.LJError) as e:
        srv.submit(7, S[:10], out)
    assert e.value.status == lj.LJ_ERR_ARG
    with pytest.raises(lj.LJError) as e:
        srv.wait(12345, 0)
    assert e.value.status == lj.LJ_ERR_ARG
    small = np.ascontiguousarray(ws[0].S[:100])
    t = srv.submit(0, small, out[:100])
    r = srv.wait(t, 60_000)
    assert r.status == lj.LJ_OK and r.count == len(oracle.sort_merge_join(ws[0].R, small))
    srv.close()


@pytest.mark.parametrize("binned_min_keys", [0, 1, 50_000])
def test_device_requests_mixed_with_host_requests(binned_min_keys):
    """Device-resident requests (no copies) interleaved with host requests,
    with the binned probe for none / all / large requests: every result
    equals the oracle's and the request's result alone."""
    import torch
    ws, ixs = _indexes()
    reqs = _requests(ws, 60, seed=23 + binned_min_keys % 7)
    cfg = lj.lj_server_default_config(1 << 28)
    cfg.slots = 4
    cfg.binned_min_keys = binned_min_keys
    srv = lj.Server(ixs, cfg)
    tickets, dev_bufs = [], []
    for q, (i, S, want, cap, out) in enumerate(reqs):
        if q % 2:
            s_dev = lj.to_device_keys(S)
            o_dev = torch.full((max(cap, 1), 2), -1, dtype=torch.int32, device="cuda")
            # The server's streams do not wait for torch's: the key copy and
            # the fill must be done before the request is submitted.
            torch.cuda.synchronize()
            dev_bufs.append((s_dev, o_dev))
            tickets.append(srv.submit_device(i, s_dev, o_dev if cap else None))
        else:
            dev_bufs.append(None)
            tickets.append(srv.submit(i, S, out if cap else None))
    print(f"[server] device requests binned_min_keys={binned_min_keys}", flush=True)
    for q, (i, S, want, cap, out) in enumerate(reqs):
        r = srv.wait(tickets[q], 60_000)
        assert r.count == len(want), (q, r.count, len(want))
        assert r.status == (lj.LJ_OK if cap >= len(want) else lj.LJ_ERR_CAPACITY)
        if dev_bufs[q] is not None:
            got = dev_bufs[q][1][:min(cap, len(want))].cpu().numpy().view(np.uint32)
        else:
            got = out[:min(cap, len(want))]
        assert np.array_equal(got, want[:cap])
    assert srv.stats.requests_done == len(reqs)
    srv.close()


def test_native_replay_driver():
    """lj_server_replay submits device requests from a native thread (all at
    once, then at spaced arrival times) and returns every result; each equals
    the oracle's."""
    import torch
    ws, ixs = _indexes()
    reqs = _requests(ws, 50, seed=31)
    srv = lj.Server(ixs, lj.lj_server_default_config(1 << 28))
    items, outs = [], []
    for i, S, want, cap, out in reqs:
        s_dev = lj.to_device_keys(S)
        o_dev = torch.full((max(cap, 1), 2), -1, dtype=torch.int32, device="cuda")
        items.append((i, s_dev, o_dev if cap else None))
        outs.append(o_dev)
    torch.cuda.synchronize()
    for arrival in (None, np.arange(len(items)) * 200_000):
        print(f"[server] replay arrival={'none' if arrival is None else 'spaced'}", flush=True)
        for o in outs:
            o.fill_(-1)
        torch.cuda.synchronize()
        res = srv.replay(items, arrival)
        for (i, S, want, cap, out), r, o in zip(reqs, res, outs):
            assert r.count == len(want)
            assert r.status == (lj.LJ_OK if cap >= len(want) else lj.LJ_ERR_CAPACITY)
            got = o[:min(cap, len(want))].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, want[:cap])
            assert r.done_ns >= r.start_ns >= r.submit_ns
    assert srv.stats.requests_done == 2 * len(items)
    srv.close()
