"""GPU parity of the HE steps around the transform (ciphertext tensor
product, fast RNS basis conversion, ModDown) against the CPU oracle, bit for
bit, through the C ABI."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P17 = si.ntt_primes(60, 17, 96)     # distinct 60-bit NTT primes for the bases
W61 = si.ntt_primes(61, 17, 80)     # primes just below 2^61 (the 4-term column groups)
Q32 = [si.Q_SMALL, 469762049, 167772161]


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def residues(seed, B, moduli, N):
    return si.poly_batch(seed, B, moduli, N)


# ---- tensor product --------------------------------------------------------------
@pytest.mark.parametrize("word,N,moduli,B", [(64, 1024, P17[:3], 2), (64, 2, P17[:1], 1), (32, 256, Q32, 3),
                                             (64, 4096, P17[:5], 1)])
def test_tensor_product_matches_oracle(ntt, word, N, moduli, B):
    import torch
    log(f"case tensor word={word} N={N} L={len(moduli)} B={B}")
    L = len(moduli)
    a = residues(50 + N, 2 * B, moduli, N).reshape(B, 2, L, N)
    b = residues(60 + N, 2 * B, moduli, N).reshape(B, 2, L, N)
    plan = ntt.Plan(N, moduli, flags=ntt.NTT_WORD32 if word == 32 else 0)
    da, db = to_dev(a, word), to_dev(b, word)
    dd = torch.zeros(B * 3 * L * N, dtype=da.dtype, device="cuda")
    plan.tensor_product(da, db, dd)
    np.testing.assert_array_equal(from_dev(dd, word).reshape(B, 3, L, N), oracle.tensor_product(a, b, moduli))


def test_tensor_product_is_the_ring_product(ntt):
    # forward NTT, tensor product, inverse NTT: each component is the ring
    # product of the input components in Z_q[x]/(x^N + 1) (schoolbook)
    import torch
    N, moduli = 1024, P17[:3]
    L = len(moduli)
    log("case tensor ring product")
    a = residues(41, 4, moduli, N)
    b = residues(42, 4, moduli, N)
    plan = ntt.Plan(N, moduli)
    da, db = to_dev(a), to_dev(b)
    dd = torch.zeros(2 * 3 * L * N, dtype=torch.int64, device="cuda")
    plan.forward(da)
    plan.forward(db)
    plan.tensor_product(da, db, dd)
    plan.inverse(dd, batch=6)
    d = from_dev(dd).reshape(2, 3, L, N)
    for ct in range(2):
        a0, a1, b0, b1 = a[2 * ct], a[2 * ct + 1], b[2 * ct], b[2 * ct + 1]
        for l, q in enumerate(moduli):
            def m(x, y):
                return oracle.negacyclic_mul(x[l], y[l], q)
            np.testing.assert_array_equal(d[ct, 0, l], m(a0, b0))
            np.testing.assert_array_equal(d[ct, 1, l], (m(a0, b1) + m(a1, b0)) % np.uint64(q))
            np.testing.assert_array_equal(d[ct, 2, l], m(a1, b1))


def test_tensor_product_rejects_bad_arguments(ntt):
    import torch
    plan = ntt.Plan(64, P17[:2])
    t = torch.zeros(3 * 2 * 64, dtype=torch.int64, device="cuda")
    assert ntt.lib().ntt_tensor_product(plan.handle, t.data_ptr(), t.data_ptr(), None, 1, None) == -1
    assert ntt.lib().ntt_tensor_product(plan.handle, t.data_ptr(), t.data_ptr(), t.data_ptr(), 0, None) == -1


# ---- basis conversion ----------------------------------------------------------
def conv_case(ntt, N, L, K, B, seed, down=False, inplace=False, primes=P17):
    import torch
    log(f"case bconv N={N} L={L} K={K} B={B} down={down} inplace={inplace} bits={primes[0].bit_length()}")
    src, dst = primes[:L], primes[L:L + K]
    x = residues(seed, B, src, N)
    conv = ntt.BaseConv(N, src, dst)
    dx = to_dev(x)
    if down:
        y = residues(seed + 1, B, dst, N)
        dy = to_dev(y)
        out = dy if inplace else torch.zeros(B * K * N, dtype=torch.int64, device="cuda")
        conv.mod_down(dx, dy, out)
        want = oracle.mod_down(x, y, src, dst)
    else:
        out = torch.zeros(B * K * N, dtype=torch.int64, device="cuda")
        conv.convert(dx, out)
        want = oracle.base_conv(x, src, dst)
    np.testing.assert_array_equal(from_dev(out).reshape(B, K, N), want)
    # the input is left as it was
    np.testing.assert_array_equal(from_dev(dx).reshape(x.shape), x)


# every register-tile size (L up to 4, 8, 12, 16, 24, 32, 48, 64), ragged
# thread counts (N/2 * B not a multiple of 256), N = 2 and non-powers of two
@pytest.mark.parametrize("N,L,K,B", [(64, 1, 3, 1), (64, 3, 1, 2), (256, 4, 4, 1), (96, 5, 7, 3),
                                     (256, 8, 24, 2), (64, 12, 5, 1), (2, 16, 16, 3), (128, 24, 8, 2),
                                     (30, 32, 4, 5), (64, 40, 3, 1), (64, 64, 2, 1), (64, 8, 64, 1)])
def test_base_conv_matches_oracle(ntt, N, L, K, B):
    conv_case(ntt, N, L, K, B, seed=100 + L * 7 + K)


@pytest.mark.parametrize("N,L,K,B,inplace", [(64, 1, 2, 1, False), (256, 8, 24, 2, False), (96, 8, 24, 1, True),
                                             (64, 24, 8, 2, True), (62, 33, 5, 3, False), (64, 64, 3, 1, False)])
def test_mod_down_matches_oracle(ntt, N, L, K, B, inplace):
    conv_case(ntt, N, L, K, B, seed=200 + L * 7 + K, down=True, inplace=inplace)


# primes just below 2^61: four-term groups, every register tile of that path,
# with and without the high-word reduction (sum of the source primes >= 2^64
# from L = 9 on)
@pytest.mark.parametrize("N,L,K,B,down", [(64, 1, 3, 2, False), (96, 4, 5, 1, True), (64, 7, 9, 2, False),
                                          (64, 8, 8, 1, True), (30, 16, 4, 3, False), (64, 29, 6, 1, True),
                                          (64, 64, 3, 1, False)])
def test_conversion_61bit_primes(ntt, N, L, K, B, down):
    conv_case(ntt, N, L, K, B, seed=400 + L, down=down, primes=W61)


def sampled_columns(N, count, seed):
    s = si.Stream(seed)
    cols = {0, 1, N - 2, N - 1}
    while len(cols) < count:
        cols.add(s.uniform_int(0, N - 1))
    return np.array(sorted(cols))


@pytest.mark.parametrize("down", [False, True])
def test_conversion_full_size_sampled(ntt, down):
    # key switching at N = 2^16: ModUp of 3 digits of 8 limbs to 24 limbs
    # (16 other ciphertext limbs + 8 special primes) and ModDown of 2
    # polynomials from 8 special primes to 24 limbs, in the launch shape the
    # benchmark times; the oracle checks 48 sampled coefficients of each
    import torch
    N, L, K, B = 1 << 16, 8, 24, (2 if down else 3)
    log(f"case bconv full size N={N} L={L} K={K} B={B} down={down}")
    src, dst = P17[:L], P17[L:L + K]
    x = residues(300, B, src, N)
    conv = ntt.BaseConv(N, src, dst)
    dx = to_dev(x)
    out = torch.zeros(B * K * N, dtype=torch.int64, device="cuda")
    cols = sampled_columns(N, 48, 301)
    if down:
        y = residues(302, B, dst, N)
        conv.mod_down(dx, to_dev(y), out)
        want = oracle.mod_down(np.ascontiguousarray(x[:, :, cols]), np.ascontiguousarray(y[:, :, cols]), src, dst)
    else:
        conv.convert(dx, out)
        want = oracle.base_conv(np.ascontiguousarray(x[:, :, cols]), src, dst)
    got = from_dev(out).reshape(B, K, N)
    np.testing.assert_array_equal(got[:, :, cols], want)
    assert (got < np.array(dst, np.uint64)[None, :, None]).all()


def test_conversion_rejects_bad_arguments(ntt):
    import torch
    conv = ntt.BaseConv(64, P17[:2], P17[2:4])
    t = torch.zeros(2 * 2 * 64 + 2, dtype=torch.int64, device="cuda")
    lib = ntt.lib()
    p = t.data_ptr()
    assert lib.ntt_base_conv(conv.handle, p + 8, p, 1, None) == -1        # misaligned
    assert lib.ntt_base_conv(conv.handle, p, p, 0, None) == -1            # empty batch
    assert lib.ntt_mod_down(conv.handle, p, None, p, 1, None) == -1       # no y
    assert lib.ntt_base_conv(None, p, p, 1, None) == -1


def test_conversion_plan_info(ntt):
    import ctypes
    conv = ntt.BaseConv(96, P17[:5], P17[5:12])
    n, l, k = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    assert ntt.lib().ntt_bconv_get_info(conv.handle, ctypes.byref(n), ctypes.byref(l), ctypes.byref(k)) == 0
    assert (n.value, l.value, k.value) == (96, 5, 7)
    assert ntt.lib().ntt_bconv_get_info(None, None, None, None) == -1
    conv.close()
    conv.close()          # closing twice is harmless
