"""ntt_forward_noalloc through the C ABI: the same spectra as ntt_forward
(and the oracle) with the library's fixed scratch array, on consecutive
calls of different sizes, and its size limit."""
import ctypes

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P17 = si.ntt_primes(60, 17, 24)


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def both_ways(ntt, plan, x, batch, stream=None):
    """(ntt_forward result, ntt_forward_noalloc result) of x on the device."""
    lib = ntt.lib()
    d_ref, d_new = to_dev(x), to_dev(x)
    assert lib.ntt_forward(plan.handle, d_ref.data_ptr(), batch, stream) == 0
    assert lib.ntt_forward_noalloc(plan.handle, d_new.data_ptr(), batch, stream) == 0
    return from_dev(d_ref).reshape(x.shape), from_dev(d_new).reshape(x.shape)


@pytest.mark.parametrize("twist", [False, True])
def test_noalloc_matches_forward_on_two_calls(ntt, twist):
    # first the headline shape (4 polynomials x 24 limbs at 2^16: 48 MiB of
    # scratch), then a smaller one on the same array
    N = 1 << 16
    plan = ntt.Plan(N, P17)
    if twist:
        plan.set_row_twist(ntt.NTT_ROW_TWIST_FWD | ntt.NTT_ROW_TWIST_INV)
    assert plan.workspace_bytes(4) == 48 << 20
    for batch, L, seed in ((4, 24, 1), (1, 3, 2)):
        log(f"case noalloc N={N} batch={batch} L={L} twist={twist}")
        small = plan if L == 24 else ntt.Plan(N, P17[:L])
        if twist and small is not plan:
            small.set_row_twist(ntt.NTT_ROW_TWIST_FWD)
        x = si.poly_batch(700 + seed, batch, P17[:L], N)
        ref, got = both_ways(ntt, small, x, batch)
        np.testing.assert_array_equal(got, ref)
        for b, l in ((0, 0), (batch - 1, L - 1)):
            np.testing.assert_array_equal(got[b, l], oracle.ntt_forward(x[b, l], P17[l]))
        if small is not plan:
            small.close()
    plan.close()


def test_noalloc_other_sizes_and_stream(ntt):
    import torch
    lib = ntt.lib()
    s = torch.cuda.Stream()
    for N, L, batch in ((1 << 17, 4, 2), (1 << 12, 5, 3), (1 << 15, 8, 2)):
        log(f"case noalloc N={N} L={L} batch={batch} on a side stream")
        plan = ntt.Plan(N, si.ntt_primes(60, 18, L))
        x = si.poly_batch(N + L, batch, plan.moduli, N)
        d = to_dev(x)
        torch.cuda.synchronize()
        assert lib.ntt_forward_noalloc(plan.handle, d.data_ptr(), batch, s.cuda_stream) == 0
        s.synchronize()
        got = from_dev(d).reshape(x.shape)
        np.testing.assert_array_equal(got, oracle.ntt_forward_batch(x, plan.moduli)[0])
        plan.close()


def test_noalloc_refuses_what_does_not_fit(ntt):
    import torch
    lib = ntt.lib()
    plan = ntt.Plan(1 << 16, P17)
    t = torch.zeros(16, dtype=torch.int64, device="cuda")
    # 8 x 24 x 2^16 words need 96 MiB: refused before anything is enqueued
    assert plan.workspace_bytes(8) > ntt.NTT_NOALLOC_SCRATCH_BYTES
    assert lib.ntt_forward_noalloc(plan.handle, t.data_ptr(), 8, None) == ntt.NTT_ERR_SCRATCH
    assert lib.ntt_forward_noalloc(plan.handle, None, 1, None) == -1
    assert lib.ntt_forward_noalloc(plan.handle, t.data_ptr(), 0, None) == -1
    assert lib.ntt_forward_noalloc(None, t.data_ptr(), 1, None) == -1
    lib.ntt_strerror.restype = ctypes.c_char_p
    assert b"scratch" in lib.ntt_strerror(ntt.NTT_ERR_SCRATCH)
    plan.close()
