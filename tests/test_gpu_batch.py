"""Batched executor (one hipGraph launch for uneven jobs) and the autotuner,
against the CPU oracle."""
import os

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


def make_jobs(seed, specs):
    """specs: list of (logN, L, op); returns host arrays, moduli lists."""
    s = si.Stream(seed)
    out = []
    for logn, L, op in specs:
        N = 1 << logn
        moduli = P18[s.uniform_int(0, 40 - L):][:L]
        x = np.stack([s.uniform_mod(q, N) for q in moduli])
        out.append((N, moduli, op, x))
    return out


def expected(job):
    N, moduli, op, x = job
    fn = oracle.ntt_forward if op == 0 else oracle.ntt_inverse
    return np.stack([fn(x[l], q) for l, q in enumerate(moduli)])


SPECS = [(4, 3, 0), (8, 1, 0), (12, 2, 0), (13, 4, 0), (14, 3, 0), (15, 2, 0), (16, 3, 0), (17, 1, 0),
         (12, 5, 1), (16, 2, 1), (10, 2, 0), (16, 1, 0), (12, 1, 0)]


@pytest.mark.parametrize("flags", [0, 1, 2, 4])
def test_batch_mixed_jobs_match_oracle(ntt, flags):
    log(f"case batch mixed flags={flags}")
    jobs = make_jobs(1, SPECS)
    tensors = [to_dev(x) for (_, _, _, x) in jobs]
    with ntt.Batch([(N, m, op, t) for (N, m, op, _), t in zip(jobs, tensors)], flags=flags) as b:
        info = b.info
        assert info["items"] == sum(L for (_, L, _) in SPECS)
        assert info["uses_graph"] == (0 if flags == 1 else 1)
        b.run()
        for job, t in zip(jobs, tensors):
            np.testing.assert_array_equal(from_dev(t).reshape(job[3].shape), expected(job))


def test_graph_replays(ntt):
    import torch
    log("case batch graph replays")
    jobs = make_jobs(2, [(12, 3, 0), (16, 2, 0), (14, 2, 1), (13, 1, 0)])
    exp = [expected(j) for j in jobs]
    tensors = [to_dev(x) for (_, _, _, x) in jobs]
    with ntt.Batch([(N, m, op, t) for (N, m, op, _), t in zip(jobs, tensors)]) as b:
        for rep in range(4):
            # the program's own eager work between replays: reload the inputs
            for (_, _, _, x), t in zip(jobs, tensors):
                t.copy_(to_dev(x))
            torch.cuda.synchronize()
            b.run()
            torch.cuda.synchronize()
            for e, t, j in zip(exp, tensors, jobs):
                np.testing.assert_array_equal(from_dev(t).reshape(j[3].shape), e, err_msg=f"replay {rep}")


def test_batch_round_trip_uneven_cfg(ntt):
    # the uneven batched shape at reduced count: N in 2^12..2^16, L in 1..32
    log("case batch uneven round trip")
    js = si.batched_jobs(count=24)
    primes = si.batched_primes()
    s = si.Stream(7)
    fwd_jobs, hosts = [], []
    for j in js:
        x = np.stack([s.uniform_mod(q, j.N) for q in primes[:j.L]])
        hosts.append(x)
    tensors = [to_dev(x) for x in hosts]
    fwd = ntt.Batch([(j.N, primes[:j.L], 0, t) for j, t in zip(js, tensors)])
    inv = ntt.Batch([(j.N, primes[:j.L], 1, t) for j, t in zip(js, tensors)])
    fwd.run()
    # spot-check forward outputs on a few limbs against the oracle
    for j, x, t in list(zip(js, hosts, tensors))[:6]:
        got = from_dev(t).reshape(x.shape)
        for l in (0, j.L - 1):
            np.testing.assert_array_equal(got[l], oracle.ntt_forward(x[l], primes[l]))
    inv.run()
    for x, t in zip(hosts, tensors):
        np.testing.assert_array_equal(from_dev(t).reshape(x.shape), x)
    fwd.close()
    inv.close()


def test_batch_argument_errors(ntt):
    import torch
    t = torch.zeros(1024, dtype=torch.int64, device="cuda")
    with pytest.raises(ntt.NttError):               # two graph forms at once
        ntt.Batch([(1024, P18[:1], 0, t)], flags=ntt.NTT_BATCH_BRANCHES | ntt.NTT_BATCH_SERIAL)
    with pytest.raises(ntt.NttError):
        ntt.Batch([(1000, P18[:1], 0, t)])          # N not a power of two
    with pytest.raises(ntt.NttError):
        ntt.Batch([(1024, [7681], 0, t)])            # 2N does not divide q-1
    with pytest.raises(ntt.NttError):
        ntt.Batch([(8, P18[:1], 0, t)])              # below the batched minimum N=16


def test_autotune_and_plan_selection(ntt, tmp_path):
    log("case autotune")
    ntt.ntt_tune_clear()
    best = ntt.ntt_autotune(1 << 16, items=96, reps=5)
    assert best["path"] in (ntt.NTT_PATH_LDS, ntt.NTT_PATH_FOURSTEP) and best["us_per_call"] > 0
    assert best["lv_col"] in (0, 4) and best["col_tile"] in (0, 32)
    # -1: the plan's default row forms (kept unless another is clearly faster)
    assert best["row_twist"] in ((-1, 0, 1, 2) if best["path"] == ntt.NTT_PATH_FOURSTEP else (-1,))
    plan = ntt.Plan(1 << 16, P18[:2])
    assert plan.variant[0] == ntt.NTT_PATH_FOURSTEP  # stored default, unchanged
    assert ntt.ntt_plan_get_variant_for(plan.handle, 48)[:2] == (best["path"], best["log_n1"])
    # the tuned variant still gives oracle results
    x = si.poly_batch(5, 48, P18[:2], 1 << 16)
    d = to_dev(x)
    plan.forward(d)
    X = from_dev(d).reshape(x.shape)
    for b in (0, 47):
        for l in (0, 1):
            np.testing.assert_array_equal(X[b, l], oracle.ntt_forward(x[b, l], P18[l]))
    f = str(tmp_path / "tune.json")
    ntt.ntt_tune_save(f)
    ntt.ntt_tune_clear()
    assert ntt.ntt_plan_get_variant_for(plan.handle, 48)[0] == ntt.NTT_PATH_FOURSTEP
    ntt.ntt_tune_load(f)
    assert ntt.ntt_plan_get_variant_for(plan.handle, 48)[:2] == (best["path"], best["log_n1"])
    ntt.ntt_tune_clear()


@pytest.mark.parametrize("logn,logn1,twist,lv,tile", [(16, 8, 3, 4, 0), (16, 7, 1, 4, 0), (17, 9, 2, 4, 0),
                                                      (14, 6, 3, 0, 0), (16, 8, 0, 4, 0), (16, 8, 3, 0, 32),
                                                      (16, 8, 3, 4, 32), (17, 9, 2, 0, 32), (17, 9, 0, 4, 32),
                                                      (14, 6, 3, 0, 32), (13, 7, 1, 0, 32)])
def test_tuned_row_form_and_values_per_thread(ntt, tmp_path, logn, logn1, twist, lv, tile):
    """A tuning table that picks the row form of each direction, 16 values per
    thread and 32 columns per tile in the column passes: a plan in automatic
    mode runs with them and still matches the oracle (forward, fused product
    + inverse, inverse)."""
    import ctypes
    log(f"case tuned row form N=2^{logn} logn1={logn1} twist={twist} lv={lv} tile={tile}")
    f = tmp_path / "arch.json"
    ntt.ntt_tune_clear()
    ntt.ntt_tune_save(str(f))
    arch = f.read_text().split('"arch": "')[1].split('"')[0]
    f.write_text('{"arch": "%s", "entries": [{"word": 64, "log_n": %d, "items_log2": 2, "path": 3, "log_n1": %d, '
                 '"exact": 0, "us": 1, "row_twist": %d, "lv_col": %d, "col_tile": %d}]}'
                 % (arch, logn, logn1, twist, lv, tile))
    ntt.ntt_tune_load(str(f))
    N, moduli = 1 << logn, P18[:2]
    try:
        plan = ntt.Plan(N, moduli)
        assert ntt.ntt_plan_get_variant_for(plan.handle, 2)[:2] == (ntt.NTT_PATH_FOURSTEP, logn1)
        assert ntt.ntt_plan_get_col_tile(plan.handle, 2) == (tile or 16)
        a = si.poly_batch(logn + twist, 2, moduli, N)
        b = si.poly_batch(logn + twist + 1, 2, moduli, N)
        da, db = to_dev(a), to_dev(b)
        plan.forward(da)
        plan.forward(db)
        A = oracle.ntt_forward_batch(a, moduli)[0]
        np.testing.assert_array_equal(from_dev(da).reshape(a.shape), A)
        dc = to_dev(np.zeros_like(a))
        plan.pointwise_inverse(da, db, dc)
        want = oracle.ntt_inverse_batch(oracle.pointwise_batch(A, oracle.ntt_forward_batch(b, moduli)[0],
                                                               moduli)[0], moduli)[0]
        np.testing.assert_array_equal(from_dev(dc).reshape(a.shape), want)
        plan.inverse(db)
        np.testing.assert_array_equal(from_dev(db).reshape(b.shape), b)
        plan.close()
    finally:
        ntt.ntt_tune_clear()
        ntt.ntt_tune_load(os.path.join(os.path.dirname(ntt.library_path()), "tune_gfx950.json"))
