"""Failure injection from the host: with NTT_FAIL_ALLOC=k the library's k-th
device or pinned-host allocation (counted from when the variable is set)
fails. Each creating call must then return NULL with NTT_ERR_NOMEM, each
other call NTT_ERR_NOMEM, with nothing launched; and once the variable is
cleared the same calls succeed and compute what the oracle computes. No
object whose call failed is used for a launch."""
import contextlib
import os

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P18 = si.ntt_primes(60, 18, 4)


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


@contextlib.contextmanager
def failing(k):
    os.environ["NTT_FAIL_ALLOC"] = str(k)
    try:
        yield
    finally:
        os.environ.pop("NTT_FAIL_ALLOC", None)


def test_plan_creation_and_first_call(ntt):
    """A 2^16 plan allocates its tables at creation and its scratch at the
    first four-step call: every k up to the first success fails cleanly."""
    N, moduli = 1 << 16, P18[:2]
    x = si.poly_batch(61, 2, moduli, N)
    want = oracle.ntt_forward_batch(x, moduli)[0]
    lib = ntt.lib()
    outcomes = []
    for k in range(1, 12):
        log(f"case allocation {k} fails: plan 2^16, forward")
        with failing(k):
            try:
                plan = ntt.Plan(N, moduli)
            except ntt.NttError as e:
                assert e.code == ntt.NTT_ERR_NOMEM, e
                outcomes.append("create")
                continue
            d = to_dev(x)
            rc = lib.ntt_forward(plan.handle, d.data_ptr(), 2, None)
        if rc == ntt.NTT_ERR_NOMEM:
            outcomes.append("call")
            np.testing.assert_array_equal(from_dev(d).reshape(x.shape), x)   # nothing ran
        else:
            assert rc == ntt.NTT_OK
            np.testing.assert_array_equal(from_dev(d).reshape(x.shape), want)
            outcomes.append("ok")
        plan.close()
        if outcomes[-1] == "ok":
            break
    assert outcomes[0] == "create" and "call" in outcomes and outcomes[-1] == "ok", outcomes


def test_fused_product_scratch(ntt):
    """ntt_polymul's workspace is its first allocation on a fresh stream."""
    import torch
    N, moduli = 1 << 16, P18[:2]
    a = si.poly_batch(62, 1, moduli, N)
    b = si.poly_batch(63, 1, moduli, N)
    A, B = oracle.ntt_forward_batch(a, moduli)[0], oracle.ntt_forward_batch(b, moduli)[0]
    want = oracle.ntt_inverse_batch(oracle.pointwise_batch(A, B, moduli)[0], moduli)[0]
    plan = ntt.Plan(N, moduli)
    lib = ntt.lib()
    da, db, dc = to_dev(a), to_dev(b), to_dev(np.zeros_like(a))
    st = torch.cuda.Stream()   # a stream the plan has no scratch for yet
    log("case allocation 1 fails: ntt_polymul workspace")
    with failing(1):
        rc = lib.ntt_polymul(plan.handle, da.data_ptr(), db.data_ptr(), dc.data_ptr(), 1, st.cuda_stream)
    assert rc == ntt.NTT_ERR_NOMEM
    rc = lib.ntt_polymul(plan.handle, da.data_ptr(), db.data_ptr(), dc.data_ptr(), 1, st.cuda_stream)
    assert rc == ntt.NTT_OK
    st.synchronize()
    np.testing.assert_array_equal(from_dev(dc).reshape(a.shape), want)
    plan.close()


def test_batch_creation(ntt):
    """Pool tables for new (q, N) pairs, bucket scratch and the descriptor
    table: a failure at any of them fails the batch alone. (The pool's pinned
    host copy of a table falls back to pageable memory, so a failure there
    does not fail the batch.)"""
    moduli = si.ntt_primes(60, 17, 3)   # pairs this process has not pooled yet
    shapes = [(1 << 12, 2), (1 << 16, 3), (1 << 14, 1)]
    xs = [si.poly_batch(70 + i, 1, moduli[:L], N)[0] for i, (N, L) in enumerate(shapes)]
    wants = [oracle.ntt_forward_batch(x[None], moduli[:L])[0][0] for (N, L), x in zip(shapes, xs)]
    outcomes = []
    for k in range(1, 13):
        log(f"case allocation {k} fails: batch of 3 polynomials")
        ts = [to_dev(x) for x in xs]
        with failing(k):
            try:
                batch = ntt.Batch([(N, moduli[:L], ntt.NTT_JOB_FORWARD, t) for (N, L), t in zip(shapes, ts)])
            except ntt.NttError as e:
                assert e.code == ntt.NTT_ERR_NOMEM, e
                outcomes.append("create")
                continue
        batch.run()
        for x, t, want in zip(xs, ts, wants):
            np.testing.assert_array_equal(from_dev(t).reshape(x.shape), want)
        batch.close()
        outcomes.append("ok")
    assert "create" in outcomes and outcomes[-1] == "ok", outcomes


def test_server_creation(ntt):
    """The arena, then each slot's device and pinned descriptor buffers."""
    N, moduli = 1 << 12, P18[:2]
    x = si.poly_batch(80, 1, moduli, N)[0]
    want = oracle.ntt_forward_batch(x[None], moduli)[0][0]
    outcomes = []
    for k in range(1, 10):
        log(f"case allocation {k} fails: server with 2 streams")
        with failing(k):
            try:
                server = ntt.Server(hbm_budget_bytes=64 << 20, n_streams=2)
            except ntt.NttError as e:
                assert e.code == ntt.NTT_ERR_NOMEM, e
                outcomes.append("create")
                continue
        a, out = to_dev(x), to_dev(np.zeros_like(x))
        t = server.submit(ntt.NTT_REQ_NTT, N, moduli, a, out)
        assert server.wait(t) == ntt.NTT_OK
        np.testing.assert_array_equal(from_dev(out).reshape(x.shape), want)
        server.close()
        outcomes.append("ok")
        break
    assert outcomes[0] == "create" and outcomes[-1] == "ok", outcomes


def test_conversion_plan_creation(ntt):
    src, dst = si.ntt_primes(60, 17, 27)[24:27], si.ntt_primes(60, 17, 24)[:4]
    outcomes = []
    for k in range(1, 6):
        log(f"case allocation {k} fails: conversion plan")
        with failing(k):
            try:
                conv = ntt.BaseConv(1 << 12, src, dst)
            except ntt.NttError as e:
                assert e.code == ntt.NTT_ERR_NOMEM, e
                outcomes.append("create")
                continue
        conv.close()
        outcomes.append("ok")
        break
    assert outcomes[0] == "create" and outcomes[-1] == "ok", outcomes


def test_autotune_allocations(ntt, tmp_path):
    """The autotuner's own plan and timing buffer: a failure at either is
    NTT_ERR_NOMEM. The process's tuning table is saved first and restored
    after, so later tests run with the table they would otherwise see."""
    ntt.Plan(1 << 12, P18[:1]).close()      # the process's table is loaded at its first plan
    saved = str(tmp_path / "tune.json")
    ntt.ntt_tune_save(saved)
    outcomes = []
    try:
        for k in range(1, 10):
            log(f"case allocation {k} fails: autotune 2^12")
            with failing(k):
                try:
                    best = ntt.ntt_autotune(1 << 12, items=8, reps=2)
                except ntt.NttError as e:
                    assert e.code == ntt.NTT_ERR_NOMEM, e
                    outcomes.append("fail")
                    continue
            assert best["us_per_call"] > 0
            outcomes.append("ok")
            break
    finally:
        ntt.ntt_tune_clear()
        ntt.ntt_tune_load(saved)
    assert outcomes[0] == "fail" and outcomes[-1] == "ok", outcomes
