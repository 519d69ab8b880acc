"""The seeded input generator: stream, residues, prime sets, job mixes."""
import numpy as np

import seeded_inputs as si


def test_vector_and_scalar_splitmix_agree():
    v = si.splitmix64(12345, 10, 50)
    assert [int(x) for x in v] == [si.splitmix64_scalar(12345, k) for k in range(10, 60)]


def test_uniform_mod_in_range_and_reproducible():
    for q in (si.Q_SMALL, si.ntt_primes(60, 17, 1)[0], 12289):
        a = si.Stream(3).uniform_mod(q, 10000)
        b = si.Stream(3).uniform_mod(q, 10000)
        np.testing.assert_array_equal(a, b)
        assert int(a.max()) < q
        # the stream is consumed in order: two draws concatenate to one
        s = si.Stream(3)
        c = np.concatenate([s.uniform_mod(q, 4000), s.uniform_mod(q, 6000)])
        np.testing.assert_array_equal(a, c)


def test_rejection_consumes_the_stream_in_order():
    # a small modulus forces rejections; the accepted values are exactly the
    # in-range shifted outputs, in stream order
    q = 12289
    shift = 64 - q.bit_length()
    raw = [si.splitmix64_scalar(5, k) >> shift for k in range(200)]
    expect = [v for v in raw if v < q][:50]
    assert [int(v) for v in si.Stream(5).uniform_mod(q, 50)] == expect


def test_poly_batch_layout():
    moduli = si.ntt_primes(60, 15, 3)
    x = si.poly_batch(1, 2, moduli, 16)
    assert x.shape == (2, 3, 16) and x.dtype == np.uint64
    s = si.Stream(1)
    assert [int(v) for v in x[0, 0]] == [int(v) for v in s.uniform_mod(moduli[0], 16)]
    assert [int(v) for v in x[0, 1]] == [int(v) for v in s.uniform_mod(moduli[1], 16)]


def test_job_mixes():
    jobs = si.batched_jobs()
    assert len(jobs) == 256
    assert {j.N for j in jobs} <= {1 << k for k in range(12, 17)}
    assert all(1 <= j.L <= 32 for j in jobs)
    tr = si.serving_trace(count=300)
    assert all(b.arrival_s > a.arrival_s for a, b in zip(tr, tr[1:]))
    assert {j.op for j in tr} == {"ntt", "polymul"}
    assert all(j.N <= 1 << 17 and 1 <= j.L <= 40 for j in tr)


def test_configs_match_the_generator():
    """configs/*.json record the workloads the tests and bench.py draw; they
    are written by seeded_inputs.configs and must not drift from it."""
    import json
    import os

    from seeded_inputs.configs import CONFIG_DIR, workload_configs
    want = workload_configs()
    files = sorted(f for f in os.listdir(CONFIG_DIR) if f.endswith(".json"))
    assert files == sorted(name + ".json" for name in want)
    for name, cfg in want.items():
        with open(os.path.join(CONFIG_DIR, name + ".json")) as fh:
            assert json.load(fh) == json.loads(json.dumps(cfg)), name
    # the primes in the files are the ones the plans are built with
    head = want["polymul_n65536_l24"]
    assert [int(q) for q in head["moduli"]] == si.workload_polymul_n16().moduli
    assert all(int(q) % (1 << 17) == 1 for q in head["moduli"])
