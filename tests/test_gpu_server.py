"""Serving loop on the GPU: results against the oracle, and each job's
result identical alone and in a concurrent mix (tolerance: 0 bits)."""
import threading
import time

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P18 = si.ntt_primes(60, 18, 40)


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def make_requests(seed, count, logn_lo=4, logn_hi=17, l_max=5):
    s = si.Stream(seed)
    reqs = []
    for i in range(count):
        N = 1 << s.uniform_int(logn_lo, logn_hi)
        L = s.uniform_int(1, l_max)
        op = s.uniform_int(0, 2)
        moduli = P18[:L]
        a = np.stack([s.uniform_mod(q, N) for q in moduli])
        b = np.stack([s.uniform_mod(q, N) for q in moduli]) if op == 2 else None
        reqs.append((op, N, moduli, a, b))
    return reqs


def reference(req):
    op, N, moduli, a, b = req
    if op == 0:
        return np.stack([oracle.ntt_forward(a[l], q) for l, q in enumerate(moduli)])
    if op == 1:
        return np.stack([oracle.ntt_inverse(a[l], q) for l, q in enumerate(moduli)])
    out = []
    for l, q in enumerate(moduli):
        A, B = oracle.ntt_forward(a[l], q), oracle.ntt_forward(b[l], q)
        out.append(oracle.ntt_inverse(oracle.pointwise(A, B, q), q))
    return np.stack(out)


def run(ntt, server, reqs, gap_s=0.0):
    bufs = []
    tickets = []
    for op, N, moduli, a, b in reqs:
        da = to_dev(a)
        db = to_dev(b) if b is not None else None
        dout = to_dev(np.zeros_like(a))
        bufs.append((da, db, dout))
    import torch
    torch.cuda.synchronize()
    for (op, N, moduli, a, b), (da, db, dout) in zip(reqs, bufs):
        tickets.append(server.submit(op, N, moduli, da, dout, b=db))
        if gap_s:
            time.sleep(gap_s)
    for t in tickets:
        assert server.wait(t, 60_000_000) == 0
    return [from_dev(dout).reshape(r[3].shape) for r, (_, _, dout) in zip(reqs, bufs)], bufs


def test_server_results_match_oracle(ntt):
    log("case server vs oracle")
    reqs = make_requests(1, 30)
    with ntt.Server(hbm_budget_bytes=1 << 30, n_streams=3, max_batch_items=64) as s:
        outs, bufs = run(ntt, s, reqs)
        st = s.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for r, o, (da, db, _) in zip(reqs, outs, bufs):
        np.testing.assert_array_equal(o, reference(r))
        np.testing.assert_array_equal(from_dev(da).reshape(r[3].shape), r[3])      # inputs untouched
        if db is not None:
            np.testing.assert_array_equal(from_dev(db).reshape(r[4].shape), r[4])


def test_alone_equals_in_mix(ntt):
    log("case server alone vs mix")
    reqs = make_requests(2, 40, logn_lo=10, logn_hi=17, l_max=8)
    with ntt.Server(hbm_budget_bytes=2 << 30, n_streams=1, max_batch_items=1) as s:
        alone = []
        for r in reqs:
            o, _ = run(ntt, s, [r])
            alone.append(o[0])
    with ntt.Server(hbm_budget_bytes=256 << 20, n_streams=4, max_batch_items=96) as s:
        mixed, _ = run(ntt, s, reqs)  # back to back: jobs queue while earlier batches run
        st = s.stats()
    assert st["batches"] < len(reqs)           # jobs shared batches
    assert st["max_inflight_batches"] >= 2     # and overlapped on the device
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a, m)


def test_in_place_and_swapped_aliasing(ntt):
    log("case server aliasing")
    N, moduli = 1 << 14, P18[:3]
    s_ = si.Stream(3)
    a = np.stack([s_.uniform_mod(q, N) for q in moduli])
    b = np.stack([s_.uniform_mod(q, N) for q in moduli])
    ref = reference((2, N, moduli, a, b))
    with ntt.Server(n_streams=2) as s:
        da, db = to_dev(a), to_dev(b)
        assert s.wait(s.submit(ntt.NTT_REQ_POLYMUL, N, moduli, da, da, b=db)) == 0   # out = a
        np.testing.assert_array_equal(from_dev(da).reshape(a.shape), ref)
        da, db = to_dev(a), to_dev(b)
        assert s.wait(s.submit(ntt.NTT_REQ_POLYMUL, N, moduli, da, db, b=db)) == 0   # out = b
        np.testing.assert_array_equal(from_dev(db).reshape(a.shape), ref)
        da = to_dev(a)
        assert s.wait(s.submit(ntt.NTT_REQ_NTT, N, moduli, da, da)) == 0             # in place
        np.testing.assert_array_equal(from_dev(da).reshape(a.shape), reference((0, N, moduli, a, None)))


def test_concurrent_submitters(ntt):
    log("case server concurrent submitters")
    reqs = make_requests(4, 24, logn_lo=8, logn_hi=15, l_max=4)
    results = {}
    with ntt.Server(n_streams=4, max_batch_items=32) as s:
        def worker(k):
            o, _ = run(ntt, s, reqs[k::3])
            results[k] = o
        ths = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    for k in range(3):
        for r, o in zip(reqs[k::3], results[k]):
            np.testing.assert_array_equal(o, reference(r))
