"""Scheduler logic of the serving loop without a GPU (NTT_SERVER_SIMULATE:
the batches complete after a modelled time and no device is touched)."""
import time

import pytest

import seeded_inputs as si

P18 = si.ntt_primes(60, 18, 8)
FAKE = 0x10000  # addresses are never dereferenced in simulate mode
MODREC = 72     # bytes of one 64-bit modulus record, stored with each (q, N) pair's tables


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
    # a POLYMUL at N = 2^16 holds the column-pass outputs of both operands,
    # beside the twiddle tables of its L (q, N) pairs
    budget = 2 * poly + L * (32 * N + MODREC) + (64 << 10)
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


def test_twiddle_tables_count_against_the_budget(ntt):
    """A job's tables (32N + 72 bytes per (q, N)) and its working memory must
    fit the budget together; tables stay resident across jobs and are
    evicted, least recently used first, when space is needed."""
    N = 1 << 17
    table = 32 * N + MODREC
    ws = 8 * N                              # four-step intermediate of one limb
    with sim(ntt, hbm_budget_bytes=ws + table - 1, n_streams=1) as s:
        with pytest.raises(ntt.NttError):   # fits the arena only without its table
            s.submit(ntt.NTT_REQ_NTT, N, P18[:1], FAKE, FAKE)
    budget = ws + 2 * table + (64 << 10)    # room for two tables beside one job
    with sim(ntt, hbm_budget_bytes=budget, n_streams=1, simulate_ns_per_item=1000.0) as s:
        for q in P18[:2]:
            assert s.wait(s.submit(ntt.NTT_REQ_NTT, N, [q], FAKE, FAKE)) == 0
        st = s.stats()
        assert st["table_uploads"] == 2 and st["table_evictions"] == 0 and st["table_bytes"] == 2 * table
        assert s.wait(s.submit(ntt.NTT_REQ_NTT, N, [P18[0]], FAKE, FAKE)) == 0   # resident: no upload
        assert s.stats()["table_uploads"] == 2
        assert s.wait(s.submit(ntt.NTT_REQ_NTT, N, [P18[2]], FAKE, FAKE)) == 0   # evicts the LRU (P18[1])
        st = s.stats()
        assert st["table_uploads"] == 3 and st["table_evictions"] == 1 and st["table_bytes"] == 2 * table
        assert st["peak_bytes"] <= budget
        assert s.wait(s.submit(ntt.NTT_REQ_NTT, N, [P18[0]], FAKE, FAKE)) == 0   # still resident
        assert s.stats()["table_uploads"] == 3


def test_many_tables_under_a_small_budget(ntt):
    """A stream of jobs over more (q, N) pairs than the budget can hold at once
    all complete: admission waits for tables to become unreferenced and
    evicts them."""
    mods = si.ntt_primes(60, 18, 8)
    with sim(ntt, hbm_budget_bytes=24 << 20, n_streams=3, max_batch_items=16, simulate_ns_per_item=200.0) as s:
        s_ = si.Stream(5)
        tickets = []
        for i in range(200):
            lg = s_.uniform_int(12, 17)
            L = s_.uniform_int(1, 3)
            op = s_.uniform_int(0, 2)
            first = s_.uniform_int(0, 8 - L)
            tickets.append(s.submit(op, 1 << lg, mods[first:first + L], FAKE, FAKE, b=FAKE))
        for t in tickets:
            assert s.wait(t) == 0
        st = s.stats()
        assert st["completed"] == 200 and st["failed"] == 0
        assert st["table_evictions"] > 0 and st["peak_bytes"] <= 24 << 20 and st["table_bytes"] <= 24 << 20


def test_admission_is_not_blocked_by_its_own_resident_tables(ntt):
    """A job whose tables are already resident but split the free space so
    that its working memory does not fit between them is still admitted
    once the device drains: working memory is placed first and any
    unreferenced table may move."""
    mods = si.serving_primes()            # 40 primes, 1 mod 2^18
    N = 1 << 14
    with sim(ntt, hbm_budget_bytes=32 << 20, n_streams=1, simulate_ns_per_item=100.0) as s:
        # an NTT job: 5 MiB of working memory, then its 40 tables (20 MiB) behind it
        assert s.wait(s.submit(ntt.NTT_REQ_NTT, N, mods, FAKE, FAKE)) == 0
        # a product over the same primes: 10 MiB of working memory and the same tables
        assert s.wait(s.submit(ntt.NTT_REQ_POLYMUL, N, mods, FAKE, FAKE, b=FAKE), 5_000_000) == 0
        st = s.stats()
        assert st["completed"] == 2 and st["peak_bytes"] <= 32 << 20
