"""NTT_DEBUG_CHECK: a plan that checks the canonical-input precondition
returns NTT_ERR_RANGE for an input word at or above its modulus, enqueues
nothing else (the data stays as it was), and computes as usual otherwise."""
import os

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P18 = si.ntt_primes(60, 18, 3)


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


@pytest.mark.parametrize("word,N", [(64, 1 << 16), (64, 1 << 12), (32, 1 << 10)])
def test_out_of_range_input_is_refused(ntt, word, N):
    moduli = P18 if word == 64 else [si.Q_SMALL, 469762049]
    log(f"case debug check word={word} N={N}")
    flags = ntt.NTT_DEBUG_CHECK | (ntt.NTT_WORD32 if word == 32 else 0)
    plan = ntt.Plan(N, moduli, flags=flags)
    lib = ntt.lib()
    x = si.poly_batch(900 + N, 2, moduli, N)
    d = to_dev(x, word)
    plan.forward(d)                                       # canonical: computed
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), oracle.ntt_forward_batch(x, moduli)[0])
    for pos, val in (((1, 1, N - 1), moduli[1]), ((0, 0, 0), moduli[0] + 5)):
        bad = x.copy()
        bad[pos] = val
        d = to_dev(bad, word)
        assert lib.ntt_forward(plan.handle, d.data_ptr(), 2, None) == ntt.NTT_ERR_RANGE
        np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), bad)   # untouched
        good = to_dev(x, word)
        out = to_dev(np.zeros_like(x), word)
        assert lib.ntt_pointwise_mul(plan.handle, good.data_ptr(), d.data_ptr(), out.data_ptr(), 2, None) == \
            ntt.NTT_ERR_RANGE
        assert lib.ntt_inverse(plan.handle, d.data_ptr(), 2, None) == ntt.NTT_ERR_RANGE
    plan.close()


def test_environment_variable_turns_it_on(ntt):
    N, moduli = 1 << 14, P18[:2]
    log("case debug check from the environment")
    x = si.poly_batch(77, 1, moduli, N)
    x[0, 1, 7] = moduli[1]
    os.environ["NTT_DEBUG_CHECK"] = "1"
    try:
        plan = ntt.Plan(N, moduli)
    finally:
        del os.environ["NTT_DEBUG_CHECK"]
    d = to_dev(x)
    assert ntt.lib().ntt_forward(plan.handle, d.data_ptr(), 1, None) == ntt.NTT_ERR_RANGE
    quiet = ntt.Plan(N, moduli)          # created without the variable: no check, no error
    assert ntt.lib().ntt_forward(quiet.handle, d.data_ptr(), 1, None) == 0
    plan.close()
    quiet.close()
