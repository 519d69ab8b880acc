"""The cyclic transform (Eq. 3 of the paper, its own setting: 32-bit primes)
on the GPU against the oracle's DIT/DIF."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu
Q32 = [si.Q_SMALL, 469762049]
P18 = si.ntt_primes(60, 18, 4)


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def brv_perm(N):
    bits = N.bit_length() - 1
    return np.array([int(format(i, f"0{bits}b")[::-1], 2) if bits else 0 for i in range(N)])


@pytest.mark.parametrize("word,logn,bitrev,variant", [
    (32, 1, False, None), (32, 3, False, None), (32, 4, False, None), (32, 10, False, None),
    (32, 10, True, None), (32, 12, False, None), (32, 14, False, None), (32, 16, False, None),
    (32, 16, True, None), (32, 17, False, None), (64, 2, False, None), (64, 9, False, None),
    (64, 13, True, None), (64, 16, False, None), (64, 12, False, (3, 6)), (64, 14, False, (2, 0))])
def test_cyclic_matches_oracle(ntt, word, logn, bitrev, variant):
    N = 1 << logn
    moduli = Q32 if word == 32 else P18[:2]
    log(f"case cyclic word={word} N={N} bitrev={bitrev} variant={variant}")
    flags = ntt.NTT_CYCLIC | (ntt.NTT_WORD32 if word == 32 else 0) | (ntt.NTT_ORDER_BITREV if bitrev else 0)
    plan = ntt.Plan(N, moduli, flags=flags)
    if variant:
        plan.set_variant(*variant)
    assert plan.psi == [oracle.omega(q, N) for q in moduli]
    x = si.poly_batch(logn + word, 2, moduli, N)
    d = to_dev(x, word)
    plan.forward(d)
    ref = np.stack([np.stack([oracle.cyclic_forward(x[b, l], q) for l, q in enumerate(moduli)]) for b in range(2)])
    if bitrev:
        ref = ref[:, :, brv_perm(N)]
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), ref)
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), x)


@pytest.mark.parametrize("word,logn,logn1,bitrev", [(32, 16, 8, False), (32, 17, 9, True), (64, 12, 6, False),
                                                   (64, 16, 8, True), (64, 16, 7, False)])
@pytest.mark.parametrize("row_twist", [True, False])
def test_cyclic_fourstep_row_forms(ntt, word, logn, logn1, bitrev, row_twist):
    N = 1 << logn
    moduli = Q32[:2] if word == 32 else P18[2:4]
    log(f"case cyclic four-step word={word} N={N} logn1={logn1} bitrev={bitrev} row_twist={row_twist}")
    flags = ntt.NTT_CYCLIC | (ntt.NTT_WORD32 if word == 32 else 0) | (ntt.NTT_ORDER_BITREV if bitrev else 0)
    plan = ntt.Plan(N, moduli, flags=flags)
    plan.set_variant(ntt.NTT_PATH_FOURSTEP, logn1)
    plan.set_row_twist(row_twist)
    x = si.poly_batch(logn + 3 * word, 2, moduli, N)
    d = to_dev(x, word)
    plan.forward(d)
    ref = np.stack([np.stack([oracle.cyclic_forward(x[b, l], q) for l, q in enumerate(moduli)]) for b in range(2)])
    if bitrev:
        ref = ref[:, :, brv_perm(N)]
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), ref)
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), x)


def test_cyclic_single_16k_u32_vs_direct_definition(ntt):
    # the paper's largest Table 1 size, sampled against the definition
    N, q = 16384, si.Q_SMALL
    log("case cyclic 16K u32 sampled direct")
    x = si.Stream(99).uniform_mod(q, N)
    plan = ntt.Plan(N, [q], flags=ntt.NTT_CYCLIC | ntt.NTT_WORD32)
    d = to_dev(x, 32)
    plan.forward(d)
    X = from_dev(d, 32)
    for k in (0, 1, 2, 4095, 8192, N - 1):
        assert int(X[k]) == oracle.cyclic_direct_coeff(x, q, k)


def test_cyclic_product_is_cyclic_convolution(ntt):
    N, q = 1024, si.Q_SMALL
    log("case cyclic convolution")
    a = si.Stream(5).uniform_mod(q, N)
    b = si.Stream(6).uniform_mod(q, N)
    plan = ntt.Plan(N, [q], flags=ntt.NTT_CYCLIC | ntt.NTT_WORD32)
    da, db = to_dev(a, 32), to_dev(b, 32)
    plan.forward(da)
    plan.forward(db)
    plan.pointwise_inverse(da, db)
    got = from_dev(da, 32)
    want = oracle.cyclic_inverse(oracle.pointwise(oracle.cyclic_forward(a, q), oracle.cyclic_forward(b, q), q), q)
    np.testing.assert_array_equal(got, want)


PAPER_PATHS = ["PAPER_DIT", "PAPER_DIF", "PAPER_PEASE", "PAPER_PEASE_NC", "PAPER_STOCKHAM"]


@pytest.mark.parametrize("path", PAPER_PATHS)
@pytest.mark.parametrize("word,logn", [(32, 1), (32, 2), (32, 6), (32, 10), (32, 12), (32, 14), (64, 3), (64, 11)])
def test_paper_variants_match_oracle(ntt, path, word, logn):
    N = 1 << logn
    moduli = Q32 if word == 32 else P18[:2]
    log(f"case paper variant {path} word={word} N={N}")
    plan = ntt.Plan(N, moduli, flags=ntt.NTT_CYCLIC | (ntt.NTT_WORD32 if word == 32 else 0))
    plan.set_variant(getattr(ntt, "NTT_PATH_" + path))
    x = si.poly_batch(logn * 3 + word, 3, moduli, N)
    d = to_dev(x, word)
    plan.forward(d)
    got = from_dev(d, word).reshape(x.shape)
    for b in range(3):
        for l, q in enumerate(moduli):
            ref = {"PAPER_PEASE": oracle.pease_forward, "PAPER_PEASE_NC": oracle.pease_forward,
                   "PAPER_STOCKHAM": oracle.stockham_forward}.get(path, oracle.cyclic_forward)(x[b, l], q)
            np.testing.assert_array_equal(got[b, l], ref)
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), x)


def test_paper_variants_need_cyclic_natural_plans(ntt):
    plan = ntt.Plan(1024, Q32[:1], flags=ntt.NTT_WORD32)          # negacyclic
    with pytest.raises(ntt.NttError):
        plan.set_variant(ntt.NTT_PATH_PAPER_DIT)
    plan = ntt.Plan(1024, Q32[:1], flags=ntt.NTT_WORD32 | ntt.NTT_CYCLIC | ntt.NTT_ORDER_BITREV)
    with pytest.raises(ntt.NttError):
        plan.set_variant(ntt.NTT_PATH_PAPER_STOCKHAM)
