"""GPU parity of the fused polynomial product (ntt_polymul) against the
oracle's schoolbook product and, bit for bit, against the composition of the
library's own forward / pointwise-inverse calls, through the C ABI."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P18 = si.ntt_primes(60, 18, 6)        # 1 mod 2^18: every N up to 2^17
Q32 = [si.Q_SMALL, 469762049, 167772161]


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def composed(ntt, plan, a, b, word):
    # the unfused path: forward both, pointwise product fused into the inverse
    da, db = to_dev(a, word), to_dev(b, word)
    plan.forward(da)
    plan.forward(db)
    plan.pointwise_inverse(da, db)
    return from_dev(da, word).reshape(a.shape)


def case(ntt, N, moduli, batch, word=64, variant=None, flags=0, seed=7):
    log(f"case polymul N={N} L={len(moduli)} batch={batch} word={word} variant={variant} flags={flags}")
    import torch
    a = si.poly_batch(seed, batch, moduli, N)
    b = si.poly_batch(seed + 1, batch, moduli, N)
    plan = ntt.Plan(N, moduli, flags=flags | (ntt.NTT_WORD32 if word == 32 else 0))
    if variant is not None:
        plan.set_variant(*variant)
    da, db = to_dev(a, word), to_dev(b, word)
    dc = torch.zeros_like(da)
    plan.polymul(da, db, dc)
    got = from_dev(dc, word).reshape(a.shape)
    np.testing.assert_array_equal(from_dev(da, word).reshape(a.shape), a)   # inputs kept
    np.testing.assert_array_equal(from_dev(db, word).reshape(b.shape), b)
    return plan, a, b, got


@pytest.mark.parametrize("N,variant", [(16, None), (1024, None), (4096, (3, 6)), (8192, (3, 6)), (8192, (3, 7)),
                                       (16384, (3, 7)), (32768, (3, 7)), (32768, (3, 8)), (65536, (3, 8)),
                                       (65536, (3, 7)), (65536, (3, 9)), (131072, (3, 8))])
def test_polymul_u64(ntt, N, variant):
    moduli = P18[:3]
    plan, a, b, got = case(ntt, N, moduli, 2, variant=variant)
    np.testing.assert_array_equal(got, composed(ntt, plan, a, b, 64))
    if N <= 4096:
        for p in range(2):
            for l, q in enumerate(moduli):
                np.testing.assert_array_equal(got[p, l], oracle.negacyclic_mul(a[p, l], b[p, l], q))
    else:
        s = si.Stream(N)
        for _ in range(6):
            p, l, k = s.uniform_int(0, 1), s.uniform_int(0, len(moduli) - 1), s.uniform_int(0, N - 1)
            assert int(got[p, l, k]) == oracle.negacyclic_coeff(a[p, l], b[p, l], moduli[l], k)


@pytest.mark.parametrize("N,variant", [(2048, None), (32768, (3, 8)), (65536, (3, 8))])
def test_polymul_u32(ntt, N, variant):
    plan, a, b, got = case(ntt, N, Q32, 2, word=32, variant=variant)
    np.testing.assert_array_equal(got, composed(ntt, plan, a, b, 32))
    s = si.Stream(N + 1)
    for _ in range(6):
        p, l, k = s.uniform_int(0, 1), s.uniform_int(0, 2), s.uniform_int(0, N - 1)
        assert int(got[p, l, k]) == oracle.negacyclic_coeff(a[p, l], b[p, l], Q32[l], k)


@pytest.mark.parametrize("N,variant", [(1024, None), (16384, (3, 7))])
def test_polymul_cyclic(ntt, N, variant):
    # a cyclic plan multiplies mod x^N - 1
    moduli = [si.Q_SMALL]
    plan, a, b, got = case(ntt, N, moduli, 1, word=32, variant=variant, flags=ntt.NTT_CYCLIC)
    np.testing.assert_array_equal(got, composed(ntt, plan, a, b, 32))
    q = moduli[0]
    x, y = a[0, 0].astype(object), b[0, 0].astype(object)
    for k in (0, 1, N // 3, N - 1):
        want = sum(x[i] * y[(k - i) % N] for i in range(N)) % q
        assert int(got[0, 0, k]) == want


def test_polymul_in_place_and_bitrev_plan(ntt):
    import torch
    N, moduli = 65536, P18[:2]
    a = si.poly_batch(31, 2, moduli, N)
    b = si.poly_batch(32, 2, moduli, N)
    plan = ntt.Plan(N, moduli, flags=ntt.NTT_ORDER_BITREV)    # order flag does not apply
    log("case polymul in place, bitrev plan")
    da, db = to_dev(a), to_dev(b)
    plan.polymul(da, db, da)
    got = from_dev(da).reshape(a.shape)
    ref = composed(ntt, ntt.Plan(N, moduli), a, b, 64)
    np.testing.assert_array_equal(got, ref)


def test_polymul_paper_variant_plan_uses_default(ntt):
    N, moduli = 4096, [si.Q_SMALL]
    plan, a, b, got = case(ntt, N, moduli, 1, word=32, variant=(ntt.NTT_PATH_PAPER_STOCKHAM, 0),
                           flags=ntt.NTT_CYCLIC)
    ref = composed(ntt, ntt.Plan(N, moduli, flags=ntt.NTT_CYCLIC | ntt.NTT_WORD32), a, b, 32)
    np.testing.assert_array_equal(got, ref)


def test_polymul_rejects_bad_arguments(ntt):
    import torch
    plan = ntt.Plan(1024, P18[:1])
    t = torch.zeros(1024, dtype=torch.int64, device="cuda")
    lib = ntt.lib()
    assert lib.ntt_polymul(plan.handle, t.data_ptr(), None, t.data_ptr(), 1, None) == -1
    assert lib.ntt_polymul(plan.handle, t.data_ptr(), t.data_ptr(), t.data_ptr(), 0, None) == -1


def test_polymul_adjacent_operands(ntt):
    # b stored right after a: the column passes of both run as one launch
    import torch
    N, moduli = 65536, P18[:3]
    x = si.poly_batch(41, 4, moduli, N)
    log("case polymul adjacent operands")
    plan = ntt.Plan(N, moduli)
    dx = to_dev(x).reshape(-1)
    half = 2 * len(moduli) * N
    dc = torch.zeros(half, dtype=torch.int64, device="cuda")
    plan.polymul(dx[:half], dx[half:], dc, batch=2)
    np.testing.assert_array_equal(from_dev(dx).reshape(x.shape), x)
    got = from_dev(dc).reshape(2, len(moduli), N)
    np.testing.assert_array_equal(got, composed(ntt, plan, x[:2], x[2:], 64))


@pytest.mark.parametrize("N,L,batch", [(2, 1, 1), (4, 2, 3), (8, 1, 2), (4096, 1, 1), (4096, 4, 5)])
def test_polymul_small_and_default_shapes(ntt, N, L, batch):
    # tiny transforms (one thread each), one limb and one pair, odd batch
    moduli = P18[:L]
    plan, a, b, got = case(ntt, N, moduli, batch, seed=N + L)
    for p in range(batch):
        for l, q in enumerate(moduli):
            if N <= 8 or (p == 0 and l == 0):
                np.testing.assert_array_equal(got[p, l], oracle.negacyclic_mul(a[p, l], b[p, l], q))
    np.testing.assert_array_equal(got, composed(ntt, plan, a, b, 64))
