"""GPU parity at the edges of what the library accepts and at the full sizes
of the uneven batch and the serving mix, against the CPU oracle, bit for bit.

* Moduli just below 2^61 (the plan's ceiling): the approximate Shoup
  quotient keeps forward values in [0, 8q), and 8q is closest to 2^64 there.
  Every kernel family runs with them: the LDS-resident transform, every
  four-step split at 2^16 and 2^17 with both quotient flavours and both row
  forms, the pointwise product, the fused product + inverse, the polynomial
  product with the spectra on chip and the tensor product. 32-bit words get
  the same treatment with primes just below 2^30.
* The uneven batch at its full size: 256 polynomials, N in 2^12..2^16, 1..32
  limbs; every (polynomial, limb) transform is compared with the oracle.
* Server requests with up to 40 limbs and N up to 2^17.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P61 = si.ntt_primes(61, 18, 6)      # the largest primes below 2^61 that are 1 mod 2^18
Q30 = si.ntt_primes(30, 18, 2)      # the largest below 2^30 that are 1 mod 2^18 (32-bit words)


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def test_edge_primes_are_at_the_ceiling():
    assert all((1 << 61) - (1 << 22) < q < (1 << 61) for q in P61[:2])
    assert all((1 << 30) - (1 << 23) < q < (1 << 30) for q in Q30)


def oracle_fwd(x, moduli):
    return oracle.ntt_forward_batch(x, moduli)[0]


def oracle_inv(x, moduli):
    return oracle.ntt_inverse_batch(x, moduli)[0]


def inputs(seed, batch, moduli, N):
    """Uniform residues, with the first polynomial set to q - 1 everywhere
    (the largest canonical input) and the second one's first limb to 0."""
    x = si.poly_batch(seed, batch, moduli, N)
    for l, q in enumerate(moduli):
        x[0, l, :] = q - 1
    if batch > 1:
        x[1, 0, :] = 0
    return x


def roundtrip(ntt, N, moduli, batch, word=64, flags=0, variant=None, exact=False, row_twist=None, seed=1):
    log(f"case edge roundtrip N={N} q0={moduli[0]:#x} batch={batch} word={word} flags={flags} "
        f"variant={variant} exact={exact} row_twist={row_twist}")
    x = inputs(seed, batch, moduli, N)
    plan = ntt.Plan(N, moduli, flags=flags | (ntt.NTT_WORD32 if word == 32 else 0))
    if variant is not None:
        plan.set_variant(*variant)
    if exact:
        plan.set_exact_quotient(True)
    if row_twist is not None:
        plan.set_row_twist(row_twist)
    d = to_dev(x, word)
    plan.forward(d)
    X = from_dev(d, word).reshape(x.shape)
    ref = oracle_fwd(x, moduli)
    if flags & ntt.NTT_ORDER_BITREV:
        bits = N.bit_length() - 1
        ref = ref[:, :, [int(format(i, f"0{bits}b")[::-1], 2) for i in range(N)]]
    np.testing.assert_array_equal(X, ref)
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), x)
    plan.close()


@pytest.mark.parametrize("logn", [1, 3, 4, 8, 12, 13, 14])
def test_61bit_lds_and_tiny_paths(ntt, logn):
    variant = (ntt.NTT_PATH_LDS, 0) if logn >= 4 else None
    roundtrip(ntt, 1 << logn, P61[:3], batch=3, variant=variant, seed=600 + logn)


@pytest.mark.parametrize("logn,logn1", [(16, 7), (16, 8), (16, 9), (17, 8), (17, 9), (14, 7), (12, 6)])
@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("row_twist", [True, False])
def test_61bit_fourstep_splits(ntt, logn, logn1, exact, row_twist):
    roundtrip(ntt, 1 << logn, P61[:2], batch=2, variant=(ntt.NTT_PATH_FOURSTEP, logn1), exact=exact,
              row_twist=row_twist, seed=610 + logn * 10 + logn1)


@pytest.mark.parametrize("logn", [12, 16])
def test_61bit_bitrev_order(ntt, logn):
    roundtrip(ntt, 1 << logn, P61[2:4], batch=2, flags=ntt.NTT_ORDER_BITREV, seed=630 + logn)


@pytest.mark.parametrize("logn,variant", [(10, None), (14, None), (16, (3, 8)), (17, (3, 9))])
def test_30bit_words_at_the_ceiling(ntt, logn, variant):
    roundtrip(ntt, 1 << logn, Q30, batch=2, word=32, variant=variant, seed=640 + logn)


@pytest.mark.parametrize("logn,variant,exact", [(12, None, False), (16, None, False), (16, (3, 8), True),
                                                (17, (3, 9), False), (14, (3, 7), True)])
@pytest.mark.parametrize("row_twist", [True, False])
def test_61bit_products(ntt, logn, variant, exact, row_twist):
    """Pointwise product, fused product + inverse and the polynomial product
    with the spectra on chip, all against the oracle's forward, product and
    inverse."""
    N, moduli = 1 << logn, P61[:3]
    log(f"case 61-bit products N={N} variant={variant} exact={exact} row_twist={row_twist}")
    plan = ntt.Plan(N, moduli)
    if variant:
        plan.set_variant(*variant)
    if exact:
        plan.set_exact_quotient(True)
    plan.set_row_twist(row_twist)
    a = inputs(650 + logn, 2, moduli, N)
    b = inputs(660 + logn, 2, moduli, N)
    A, B = oracle_fwd(a, moduli), oracle_fwd(b, moduli)
    AB = oracle.pointwise_batch(A, B, moduli)[0]
    want = oracle_inv(AB, moduli)
    da, db = to_dev(a), to_dev(b)
    plan.forward(da)
    plan.forward(db)
    np.testing.assert_array_equal(from_dev(da).reshape(a.shape), A)
    dc = to_dev(np.zeros_like(a))
    plan.pointwise(da, db, dc)
    np.testing.assert_array_equal(from_dev(dc).reshape(a.shape), AB)
    plan.pointwise_inverse(da, db, dc)
    np.testing.assert_array_equal(from_dev(dc).reshape(a.shape), want)
    # the product with the spectra on chip, from the coefficient inputs
    da, db, dc = to_dev(a), to_dev(b), to_dev(np.zeros_like(a))
    plan.polymul(da, db, dc)
    np.testing.assert_array_equal(from_dev(dc).reshape(a.shape), want)
    np.testing.assert_array_equal(from_dev(da).reshape(a.shape), a)
    if logn <= 12:
        for l, q in enumerate(moduli):
            np.testing.assert_array_equal(want[1, l], oracle.negacyclic_mul(a[1, l], b[1, l], q))
    plan.close()


def test_61bit_tensor_product(ntt):
    import torch
    N, moduli, B = 4096, P61[:3], 2
    L = len(moduli)
    log("case 61-bit tensor product")
    a = inputs(670, 2 * B, moduli, N).reshape(B, 2, L, N)
    b = inputs(671, 2 * B, moduli, N).reshape(B, 2, L, N)
    plan = ntt.Plan(N, moduli)
    da, db = to_dev(a), to_dev(b)
    dd = torch.zeros(B * 3 * L * N, dtype=torch.int64, device="cuda")
    plan.tensor_product(da, db, dd)
    np.testing.assert_array_equal(from_dev(dd).reshape(B, 3, L, N), oracle.tensor_product(a, b, moduli))


# ---------------------------------------------------------------- full sizes
def _uneven_batch():
    jobs = si.batched_jobs()
    primes = si.batched_primes()
    s = si.Stream(si.BASE_SEED + 30)
    hosts = [np.stack([s.uniform_mod(q, j.N) for q in primes[:j.L]]) for j in jobs]
    return jobs, primes, hosts


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_uneven_batch_full_size_every_item(ntt, flags):
    """256 polynomials (4100 transforms, about 105 M coefficients): the
    forward batch (one graph launch, or eager launches with flags = 1) against
    the oracle on every (polynomial, limb), then the inverse batch back to the
    input."""
    jobs, primes, hosts = _uneven_batch()
    log(f"case uneven batch full size flags={flags}: {len(jobs)} polys, {sum(j.L for j in jobs)} NTTs")
    assert len(jobs) == 256
    tensors = [to_dev(x) for x in hosts]
    fwd = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_FORWARD, t) for j, t in zip(jobs, tensors)], flags=flags)
    inv = ntt.Batch([(j.N, primes[:j.L], ntt.NTT_JOB_INVERSE, t) for j, t in zip(jobs, tensors)], flags=flags)
    fwd.run()
    bad = []
    for i, (j, x, t) in enumerate(zip(jobs, hosts, tensors)):
        got = from_dev(t).reshape(x.shape)
        want = oracle_fwd(x[None], primes[:j.L])[0]
        if not np.array_equal(got, want):
            bad.append((i, j.N, j.L))
    assert not bad, f"forward differs from the oracle on jobs {bad[:8]}"
    inv.run()
    for i, (x, t) in enumerate(zip(hosts, tensors)):
        np.testing.assert_array_equal(from_dev(t).reshape(x.shape), x, err_msg=f"job {i}")
    fwd.close()
    inv.close()


def test_server_requests_up_to_40_limbs(ntt):
    """Serving mix at its full limb range: NTT, INTT and product requests with
    N up to 2^17 and up to 40 limbs, admitted together under a budget that
    forces several batches."""
    import torch
    primes = si.serving_primes()
    specs = [(0, 17, 40), (2, 17, 40), (1, 16, 40), (2, 16, 33), (0, 12, 40), (2, 12, 40), (0, 15, 27),
             (2, 14, 38), (1, 13, 40), (0, 17, 1), (2, 13, 19)]
    s = si.Stream(si.BASE_SEED + 41)
    reqs = []
    for op, logn, L in specs:
        N = 1 << logn
        moduli = primes[:L]
        a = np.stack([s.uniform_mod(q, N) for q in moduli])[None]
        b = np.stack([s.uniform_mod(q, N) for q in moduli])[None] if op == 2 else None
        reqs.append((op, N, moduli, a, b))
    log(f"case server up to 40 limbs: {len(reqs)} requests")
    with ntt.Server(hbm_budget_bytes=512 << 20, n_streams=3, max_batch_items=256) as srv:
        bufs = []
        for op, N, moduli, a, b in reqs:
            da, dout = to_dev(a), to_dev(np.zeros_like(a))
            db = to_dev(b) if b is not None else None
            bufs.append((da, db, dout))
        torch.cuda.synchronize()
        tickets = [srv.submit(op, N, moduli, da, dout, b=db)
                   for (op, N, moduli, _, _), (da, db, dout) in zip(reqs, bufs)]
        for t in tickets:
            assert srv.wait(t, 120_000_000) == 0
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for (op, N, moduli, a, b), (_, _, dout) in zip(reqs, bufs):
        if op == 0:
            want = oracle_fwd(a, moduli)
        elif op == 1:
            want = oracle_inv(a, moduli)
        else:
            prod = oracle.pointwise_batch(oracle_fwd(a, moduli), oracle_fwd(b, moduli), moduli)[0]
            want = oracle_inv(prod, moduli)
        np.testing.assert_array_equal(from_dev(dout).reshape(a.shape), want,
                                      err_msg=f"op={op} N={N} L={len(moduli)}")


@pytest.mark.parametrize("flags", [0, 2])
def test_61bit_batch_jobs(ntt, flags):
    """Batch jobs whose moduli reach 2^61 (the narrow range) beside jobs of
    60-bit primes (the wide one), forward and inverse, against the oracle."""
    P60 = si.ntt_primes(60, 18, 4)
    s = si.Stream(si.BASE_SEED + 51)
    specs = [(12, P61[:3], 0), (16, P61[:2], 0), (17, P61[:1], 1), (14, P60[:3], 0), (16, P60[:2] + P61[:1], 0),
             (13, P61[:2], 1), (10, P61[:2], 0)]
    jobs = []
    for logn, moduli, op in specs:
        N = 1 << logn
        jobs.append((N, moduli, op, np.stack([s.uniform_mod(q, N) for q in moduli])))
    log(f"case 61-bit batch jobs flags={flags}")
    tensors = [to_dev(x) for (_, _, _, x) in jobs]
    with ntt.Batch([(N, m, op, t) for (N, m, op, _), t in zip(jobs, tensors)], flags=flags) as b:
        b.run()
        for (N, m, op, x), t in zip(jobs, tensors):
            want = (oracle_fwd if op == 0 else oracle_inv)(x[None], m)[0]
            np.testing.assert_array_equal(from_dev(t).reshape(x.shape), want, err_msg=f"N={N} op={op}")
