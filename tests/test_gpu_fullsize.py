"""Full-size parity on the lognormal / Zipf workload (2e8 x 2e8, 2^20 leaves),
probed the way the benchmark probes it (FP32 leaves, synchronous probe).

The oracle's full sort-merge is too slow on the host at this size, so the
output is checked by properties that pin it exactly:
  * every emitted pair matches (S[s] == R[r]) and pairs are in strictly
    increasing (s, r) order, so no pair repeats;
  * R is duplicate-free, so P holds one pair per hit, and the generator
    draws exactly 1.8e8 hits (misses are rejected until absent from R):
    |output| == 1.8e8 together with the two facts above means output == P;
  * for 200,000 sampled outer keys the oracle's equal_range gives the same
    match (or none) as the output.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2111_08824_amd import lj

pytestmark = pytest.mark.gpu


def test_lognormal_zipf_200m_full_size():
    import torch
    print("[fullsize] generating lognormal-zipf-200M", flush=True)
    w = workloads.c2_lognormal_zipf()
    print("[fullsize] building index (fp32 leaves, 2^20)", flush=True)
    ix = lj.lj_build_rmi(w.R, w.leaves, lj.LJ_LEAF_FP32)
    assert lj.lj_self_check(ix) == 0
    s = lj.to_device_keys(w.S)
    out = torch.empty((len(w.S), 2), dtype=torch.int32, device="cuda")
    print("[fullsize] probing", flush=True)
    st, cnt = lj.lj_probe_join(ix, s, out)
    assert st == lj.LJ_OK
    assert cnt == w.expected_count == 180_000_000
    P = out[:cnt].cpu().numpy().view(np.uint32)
    del out, s
    si = P[:, 0].astype(np.int64)
    ri = P[:, 1].astype(np.int64)
    assert np.all(np.diff(si) > 0)
    assert np.array_equal(w.S[si], w.R[ri])
    rng = np.random.default_rng(1)
    sample = rng.choice(len(w.S), 200_000, replace=False)
    first, count = oracle.equal_range(w.R, w.S[sample])
    pos = np.searchsorted(si, sample)
    pos_c = np.minimum(pos, len(si) - 1)
    emitted = si[pos_c] == sample
    assert np.array_equal(emitted, count == 1)
    assert np.array_equal(ri[pos_c][emitted], first[emitted].astype(np.int64))
