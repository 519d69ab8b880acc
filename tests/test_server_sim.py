"""Scheduler logic of the serving loop without a GPU (NTT_SERVER_SIMULATE:
the batches complete after a modelled time and no device is touched)."""
import time

import pytest

import seeded_inputs as si

P18 = si.ntt_primes(60, 18, 8)
FAKE = 0x10000  # addresses are never dereferenced in simulate mode


@pytest.fixture(scope="module")
def ntt():
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def sim(ntt, **kw):
    kw.setdefault("flags", ntt.NTT_SERVER_SIMULATE)
    return ntt.Server(**kw)


def test_all_jobs_complete_and_stats(ntt):
    with sim(ntt, n_streams=2, simulate_ns_per_item=2000.0) as s:
        tickets = [s.submit(ntt.NTT_REQ_NTT if i % 3 else ntt.NTT_REQ_POLYMUL, 1 << (12 + i % 4), P18[:1 + i % 4],
                            FAKE, FAKE, b=FAKE) for i in range(40)]
        for t in tickets:
            assert s.wait(t) == 0
        st = s.stats()
        assert st["submitted"] == st["completed"] == 40 and st["failed"] == 0
        want = sum((3 if i % 3 == 0 else 1) * (1 + i % 4) for i in range(40))
        assert st["ntts"] == want
        assert st["p50_us"] <= st["p99_us"] <= st["max_us"]
        assert 1 <= st["max_inflight_batches"] <= 2
        assert st["queued"] == 0


def test_overlapping_batches_use_several_streams(ntt):
    with sim(ntt, n_streams=4, max_batch_items=8, simulate_ns_per_item=100000.0) as s:
        tickets = [s.submit(ntt.NTT_REQ_NTT, 4096, P18[:4], FAKE, FAKE) for _ in range(16)]
        for t in tickets:
            assert s.wait(t) == 0
        st = s.stats()
        assert st["max_inflight_batches"] == 4
        assert st["batches"] >= 8          # at most 8 items (2 jobs) per batch


def test_budget_admission_and_rejection(ntt):
    N, L = 1 << 16, 4
    poly = L * N * 8
    # a POLYMUL at N = 2^16 holds the column-pass outputs of both operands
    budget = 2 * poly
    with sim(ntt, hbm_budget_bytes=budget, n_streams=4, simulate_ns_per_item=50000.0) as s:
        with pytest.raises(ntt.NttError) as e:
            s.submit(ntt.NTT_REQ_POLYMUL, N, P18[:L + 1], FAKE, FAKE, b=FAKE)   # > budget
        assert e.value.code == -6
        tickets = [s.submit(ntt.NTT_REQ_POLYMUL, N, P18[:L], FAKE, FAKE, b=FAKE) for _ in range(6)]
        for t in tickets:
            assert s.wait(t) == 0
        st = s.stats()
        assert st["peak_bytes"] <= budget
        assert st["max_inflight_batches"] == 1     # only one such job fits at a time
        assert st["admission_stalls"] >= 1
        assert st["rejected"] == 1


def test_timeout_and_unknown_ticket(ntt):
    with sim(ntt, n_streams=1, simulate_ns_per_item=2e6) as s:   # 2 ms per item
        t = s.submit(ntt.NTT_REQ_NTT, 4096, P18[:8], FAKE, FAKE)  # ~16 ms
        assert s.wait(t, 0) == -9
        assert s.wait(t, 10_000_000) == 0
        assert s.wait(t, 0) == -8          # forgotten after a successful wait
        assert s.wait(12345, 0) == -8


def test_fifo_order_under_a_single_slot(ntt):
    with sim(ntt, n_streams=1, max_batch_items=1, simulate_ns_per_item=200000.0) as s:
        tickets = [s.submit(ntt.NTT_REQ_INTT, 256, P18[:1], FAKE, FAKE) for _ in range(6)]
        done_order = []
        pending = list(tickets)
        while pending:
            for t in list(pending):
                if s.wait(t, 0) == 0:
                    done_order.append(t)
                    pending.remove(t)
            time.sleep(0.0002)
        assert done_order == tickets


def test_argument_errors(ntt):
    with sim(ntt) as s:
        with pytest.raises(ntt.NttError):
            s.submit(ntt.NTT_REQ_NTT, 1000, P18[:1], FAKE, FAKE)        # N
        with pytest.raises(ntt.NttError):
            s.submit(ntt.NTT_REQ_NTT, 8, P18[:1], FAKE, FAKE)           # below 16
        with pytest.raises(ntt.NttError):
            s.submit(ntt.NTT_REQ_NTT, 1024, [7681], FAKE, FAKE)         # modulus
        with pytest.raises(ntt.NttError):
            s.submit(ntt.NTT_REQ_POLYMUL, 1024, P18[:1], FAKE, FAKE)    # missing b
    with pytest.raises(ntt.NttError):
        ntt.Server(n_streams=0, flags=ntt.NTT_SERVER_SIMULATE)


def test_destroy_drains_queued_work(ntt):
    s = sim(ntt, n_streams=1, simulate_ns_per_item=20000.0)
    for _ in range(10):
        s.submit(ntt.NTT_REQ_NTT, 1024, P18[:2], FAKE, FAKE)
    s.close()   # returns only after the queue is empty


class _FakeTensor:
    """Looks like a GPU tensor to the binding's checks; never dereferenced."""

    def __init__(self, numel, cuda=True, width=8):
        self._n, self.is_cuda, self._w = numel, cuda, width

    def numel(self):
        return self._n

    def element_size(self):
        return self._w

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return FAKE


def test_undersized_buffers_are_refused_before_submit(ntt):
    """The binding checks every buffer of a request against L*N 64-bit words
    before the C call: nothing reaches the server (its counters stay at 0)."""
    N, mods = 1 << 12, P18[:3]
    with sim(ntt, n_streams=1) as s:
        s.simulate = False  # check as a real server would
        ok = _FakeTensor(3 * N)
        bad = [(_FakeTensor(3 * N - 1), ok, None, ntt.NTT_REQ_NTT),      # a too small
               (ok, _FakeTensor(N), None, ntt.NTT_REQ_INTT),              # out too small
               (ok, ok, _FakeTensor(2 * N), ntt.NTT_REQ_POLYMUL),         # b too small
               (ok, ok, None, ntt.NTT_REQ_POLYMUL),                       # product without b
               (_FakeTensor(3 * N, cuda=False), ok, None, ntt.NTT_REQ_NTT),
               (_FakeTensor(3 * N, width=4), ok, None, ntt.NTT_REQ_NTT),
               (FAKE, ok, None, ntt.NTT_REQ_NTT)]                         # a bare address
        for a, out, b, op in bad:
            with pytest.raises(ValueError):
                s.submit(op, N, mods, a, out, b=b)
            with pytest.raises(ValueError):
                s.make_request(op, N, mods, a, out, b=b)
        assert s.stats()["submitted"] == 0
        s.simulate = True
        t = s.submit(ntt.NTT_REQ_POLYMUL, N, mods, ok, ok, b=ok)
        assert s.wait(t) == 0
