"""The batched (many indexes, one replayed plan) and served (resident
indexes, continuous batching) probes at their full stated shapes, checked
element by element against the oracle.

  * multi-index-64: 64 indexes of 1e4..5e7 keys (log-uniform; uniform,
    lognormal and seq_h shapes), one batch of 1e3..1e7 outer keys each
    (log-uniform, 50% hits), run through the autotuned plan the benchmark
    times (HIP graph replay) and through a plan that probes batches of 2^20
    keys or more binned;
  * serving-8x50M: 8 resident indexes of 5e7 keys, 240 requests of
    256..4M keys (log-uniform) over them, half with host buffers and half
    with device buffers, through the default served configuration, one
    that probes requests of 2^20 keys or more binned, and the default one
    over gapped RMIs (4 slots per key) of the same relations.

Indexes use the radix root and FP32 leaves, as the benchmark's do.

Every inner relation here is duplicate-free, so P is given element by
element by the oracle's equal_range (tests/exact_pairs.py).
"""
import numpy as np
import pytest

import workloads
from exact_pairs import expected_pairs_unique
from paper_2111_08824_amd import lj

pytestmark = pytest.mark.gpu


def test_multi_index_64_full_shape():
    import torch
    print("[fullshape] generating multi-index-64", flush=True)
    ws = workloads.multi_index_batches(k=64)
    items = []
    for w in ws:
        ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32 | lj.LJ_ROOT_RADIX)  # as benchmarked
        s = lj.to_device_keys(w.S)
        out = torch.empty((max(1, len(w.S)), 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        items.append((w, ix, s, out, cnt))
    print(f"[fullshape] {sum(len(w.R) for w in ws)} inner, {sum(len(w.S) for w in ws)} "
          "outer keys; computing the expected pairs", flush=True)
    want = [expected_pairs_unique(w.R, w.S) for w in ws]
    for w, p in zip(ws, want):
        assert len(p) == w.expected_count
    batches = [(ix, s, out, cnt) for _, ix, s, out, cnt in items]
    tuned = lj.lj_batch_autotune(batches)
    print("[fullshape] tuned", tuned.as_dict(), flush=True)
    binned = lj.lj_batch_default_tuning()
    binned.branches = 8
    binned.binned_min_keys = 1 << 20
    for name, t in (("autotuned", tuned), ("binned from 2^20", binned)):
        plan = lj.BatchPlan(batches, t)
        for rep in range(2):
            print(f"[fullshape] plan {name}, replay {rep}", flush=True)
            for *_, out, cnt in items:
                out.fill_(-1)
                cnt.fill_(-7)
            plan.run()
            torch.cuda.synchronize()
            for (w, _, _, out, cnt), p in zip(items, want):
                got_n = int(cnt.item())
                assert got_n == len(p), (w.name, got_n, len(p))
                got = out[:got_n].cpu().numpy().view(np.uint32)
                assert np.array_equal(got, p), w.name
        plan.close()


def test_serving_8x50m_full_shape():
    import torch
    print("[fullshape] generating the 8 resident indexes", flush=True)
    ws = workloads.resident_indexes()
    flags = lj.LJ_LEAF_FP32 | lj.LJ_ROOT_RADIX  # as the serving benchmark builds them
    ixs = [lj.lj_build_rmi(w.R, w.leaves, flags) for w in ws]
    gixs = [lj.lj_build_gapped_rmi(w.R, w.leaves, 4, flags) for w in ws]
    rng = np.random.default_rng(13)
    max_m = 4 << 20
    reqs = []
    for q in range(240):
        i = int(rng.integers(0, len(ws)))
        m = int(np.exp(rng.uniform(np.log(256), np.log(max_m))))
        a = int(rng.integers(0, len(ws[i].S) - m))
        reqs.append((i, a, m, q % 2 == 1))
    print(f"[fullshape] 240 requests, {sum(r[2] for r in reqs)} outer keys; computing the "
          "expected pairs", flush=True)
    want = [expected_pairs_unique(ws[i].R, ws[i].S[a:a + m]) for i, a, m, _ in reqs]
    s_dev = [lj.to_device_keys(w.S) for w in ws]
    torch.cuda.synchronize()
    budget = 24 << 30
    served = lj.lj_server_default_config(budget)
    binned = lj.lj_server_default_config(budget)
    binned.binned_min_keys = 1 << 20
    for name, cfg, idx in (("served", served, ixs), ("served, binned from 2^20", binned, ixs),
                           ("served, gapped RMIs", served, gixs)):
        print(f"[fullshape] server {name}", flush=True)
        srv = lj.Server(idx, cfg)
        tickets, outs = [], []
        for i, a, m, dev in reqs:
            if dev:
                out = torch.full((m, 2), -1, dtype=torch.int32, device="cuda")
                torch.cuda.synchronize()
                tickets.append(srv.submit_device(i, s_dev[i][a:a + m], out))
            else:
                out = np.full((m, 2), 0xFFFFFFFF, dtype=np.uint32)
                tickets.append(srv.submit(i, np.ascontiguousarray(ws[i].S[a:a + m]), out))
            outs.append(out)
        for q, (t, out, p) in enumerate(zip(tickets, outs, want)):
            r = srv.wait(t)
            assert r.status == lj.LJ_OK, (q, r.status)
            assert r.count == len(p), (q, r.count, len(p))
            got = out[:r.count]
            got = got.cpu().numpy().view(np.uint32) if reqs[q][3] else got
            assert np.array_equal(got, p), q
        st = srv.stats
        print(f"[fullshape] {name}: {st.batches} batches, largest {st.max_batch_size} "
              "requests", flush=True)
        assert st.requests_done == len(reqs)
        srv.close()
