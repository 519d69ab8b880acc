"""GPU parity: the HIP kernels (through the C ABI) against the CPU oracle.

Integer results must match bit for bit. Inputs come from the seeded
generator; each test logs its case before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import from_dev, log, to_dev

pytestmark = pytest.mark.gpu

P18 = si.ntt_primes(60, 18, 40)      # 1 mod 2^18: every N up to 2^17
P15 = si.ntt_primes(60, 15, 8)
P17 = si.ntt_primes(60, 17, 24)
Q32 = [si.Q_SMALL, 469762049, 167772161]   # < 2^30, 1 mod 2^25


@pytest.fixture(scope="module")
def ntt():
    import torch
    assert torch.cuda.is_available()
    import paper_2405_11353_amd as ntt
    ntt.lib()
    return ntt


def oracle_fwd(x, moduli):
    y, _ = oracle.ntt_forward_batch(x, moduli)
    return y


def oracle_inv(x, moduli):
    y, _ = oracle.ntt_inverse_batch(x, moduli)
    return y


def brv_perm(N):
    bits = N.bit_length() - 1
    return np.array([int(format(i, f"0{bits}b")[::-1], 2) if bits else 0 for i in range(N)])


def run_roundtrip(ntt, N, moduli, batch, word=64, flags=0, variant=None, seed=1, exact=False, row_twist=None):
    log(f"case N={N} L={len(moduli)} batch={batch} word={word} flags={flags} variant={variant} exact={exact} "
        f"row_twist={row_twist}")
    x = si.poly_batch(seed, batch, moduli, N)
    plan = ntt.Plan(N, moduli, flags=flags | (ntt.NTT_WORD32 if word == 32 else 0))
    if variant is not None:
        plan.set_variant(*variant)
    if exact:
        plan.set_exact_quotient(True)
    if row_twist is not None:
        plan.set_row_twist(row_twist)
    assert plan.psi == [oracle.psi(q, N) for q in moduli]
    d = to_dev(x, word)
    plan.forward(d)
    X = from_dev(d, word).reshape(x.shape)
    ref = oracle_fwd(x, moduli)
    if flags & ntt.NTT_ORDER_BITREV:
        ref = ref[:, :, brv_perm(N)]
    np.testing.assert_array_equal(X, ref)
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d, word).reshape(x.shape), x)
    plan.close()


@pytest.mark.parametrize("logn", list(range(1, 15)))
def test_default_path_u64(ntt, logn):
    run_roundtrip(ntt, 1 << logn, P18[:3], batch=3 if logn < 12 else 2, seed=logn)


@pytest.mark.parametrize("logn", [1, 3, 4, 7, 10, 12, 14, 15])
def test_default_path_u32(ntt, logn):
    run_roundtrip(ntt, 1 << logn, Q32, batch=2, word=32, seed=100 + logn)


# every (log2 N1, log2 N2) pair in 6..9 x 6..9 that N <= 2^17 allows
@pytest.mark.parametrize("logn,logn1", [(12, 6), (13, 6), (13, 7), (14, 6), (14, 7), (14, 8), (15, 6), (15, 7),
                                        (15, 8), (15, 9), (16, 7), (16, 8), (16, 9), (17, 8), (17, 9)])
@pytest.mark.parametrize("bitrev", [False, True])
@pytest.mark.parametrize("row_twist", [True, False, None])
def test_fourstep_splits_u64(ntt, logn, logn1, bitrev, row_twist):
    run_roundtrip(ntt, 1 << logn, P18[3:5], batch=2, flags=ntt.NTT_ORDER_BITREV if bitrev else 0,
                  variant=(ntt.NTT_PATH_FOURSTEP, logn1), seed=logn * 10 + logn1, row_twist=row_twist)


@pytest.mark.parametrize("logn,logn1", [(12, 6), (14, 8), (16, 8), (17, 8), (17, 9)])
@pytest.mark.parametrize("row_twist", [True, False])
def test_fourstep_u32(ntt, logn, logn1, row_twist):
    run_roundtrip(ntt, 1 << logn, Q32[:2], batch=2, word=32, variant=(ntt.NTT_PATH_FOURSTEP, logn1), seed=7,
                  row_twist=row_twist)


@pytest.mark.parametrize("logn", [4, 9, 12, 14])
def test_lds_path_bitrev(ntt, logn):
    run_roundtrip(ntt, 1 << logn, P18[:2], batch=2, flags=ntt.NTT_ORDER_BITREV,
                  variant=(ntt.NTT_PATH_LDS, 0), seed=logn + 50)


@pytest.mark.parametrize("logn", [12, 13, 14])
def test_lds_path_large(ntt, logn):
    run_roundtrip(ntt, 1 << logn, P18[5:7], batch=3, variant=(ntt.NTT_PATH_LDS, 0), seed=logn + 60)


@pytest.mark.parametrize("logn", [14, 16])
@pytest.mark.parametrize("row_twist", [True, False])
def test_exact_quotient_variant(ntt, logn, row_twist):
    run_roundtrip(ntt, 1 << logn, P18[:2], batch=2, variant=(ntt.NTT_PATH_FOURSTEP, logn // 2), exact=True,
                  seed=logn + 70, row_twist=row_twist)


@pytest.mark.parametrize("logn,logn1,bitrev", [(12, 6, False), (16, 8, False), (16, 8, True), (17, 9, False)])
def test_row_forms_agree_and_stages_mix(ntt, logn, logn1, bitrev):
    """Every row-pass setting gives the same spectra, and a stage run in one
    setting composes with the other stage run in another (the forward
    intermediate is the same column pass output; the column pass reduces either
    inverse intermediate). One plan, switched between the stages: the
    natural-order intermediate lives in the plan's scratch."""
    N, moduli = 1 << logn, P18[6:9]
    log(f"case row forms N={N} logn1={logn1} bitrev={bitrev}")
    plan = ntt.Plan(N, moduli, flags=ntt.NTT_ORDER_BITREV if bitrev else 0)
    plan.set_variant(ntt.NTT_PATH_FOURSTEP, logn1)
    x = si.poly_batch(logn + 400, 3, moduli, N)
    ref = oracle_fwd(x, moduli)
    if bitrev:
        ref = ref[:, :, brv_perm(N)]
    F, I = ntt.NTT_ROW_TWIST_FWD, ntt.NTT_ROW_TWIST_INV
    for fwd0, fwd1, inv0, inv1 in ((0, F, 0, I), (F, 0, I, 0), (F | I, F, I, 0), (0, 0, 0, I)):
        d = to_dev(x)
        plan.set_row_twist(fwd0)
        plan.forward_stage(d, 0)
        plan.set_row_twist(fwd1)
        plan.forward_stage(d, 1)
        np.testing.assert_array_equal(from_dev(d).reshape(x.shape), ref)
        plan.set_row_twist(inv0)
        plan.inverse_stage(d, 0)
        plan.set_row_twist(inv1)
        plan.inverse_stage(d, 1)
        np.testing.assert_array_equal(from_dev(d).reshape(x.shape), x)
    plan.close()


def test_single_ntt_u32_vs_direct(ntt):
    # one negacyclic NTT+INTT at N=1024, q=998244353, against the O(N^2) definition
    N, q = 1024, si.Q_SMALL
    log("case single u32 N=1024 vs direct definition")
    x = si.Stream(si.BASE_SEED).uniform_mod(q, N)
    plan = ntt.Plan(N, [q], flags=ntt.NTT_WORD32)
    d = to_dev(x, 32)
    plan.forward(d)
    np.testing.assert_array_equal(from_dev(d, 32), oracle.ntt_direct(x, q))
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d, 32), x)


def test_ciphertext_n14(ntt):
    w = si.workload_ct_n14()
    log(f"case {w.name}")
    x = si.poly_batch(w.seed, w.batch, w.moduli, w.N)
    plan = ntt.Plan(w.N, w.moduli)
    d = to_dev(x)
    plan.forward(d)
    np.testing.assert_array_equal(from_dev(d).reshape(x.shape), oracle_fwd(x, w.moduli))
    plan.inverse(d)
    np.testing.assert_array_equal(from_dev(d).reshape(x.shape), x)


def test_pointwise(ntt):
    for word, moduli, N in ((64, P17[:5], 4096), (32, Q32, 2048)):
        log(f"case pointwise word={word} N={N}")
        a = si.poly_batch(3, 2, moduli, N)
        b = si.poly_batch(4, 2, moduli, N)
        plan = ntt.Plan(N, moduli, flags=ntt.NTT_WORD32 if word == 32 else 0)
        da, db = to_dev(a, word), to_dev(b, word)
        dc = to_dev(np.zeros_like(a), word)
        plan.pointwise(da, db, dc)
        ref, _ = oracle.pointwise_batch(a, b, moduli)
        np.testing.assert_array_equal(from_dev(dc, word).reshape(a.shape), ref)
        plan.pointwise(da, db)   # in place into a
        np.testing.assert_array_equal(from_dev(da, word).reshape(a.shape), ref)


def test_pointwise_edge_values(ntt):
    q = P17[0]
    N = 64
    vals = np.array([0, 1, 2, q - 1, q - 2, q // 2, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, q // 3], np.uint64)
    a = np.resize(vals, N).reshape(1, 1, N)
    b = np.resize(vals[::-1], N).reshape(1, 1, N)
    log("case pointwise edge values")
    plan = ntt.Plan(N, [q])
    da, db = to_dev(a), to_dev(b)
    plan.pointwise(da, db, da)
    np.testing.assert_array_equal(from_dev(da).ravel(), [int(x) * int(y) % q for x, y in zip(a.ravel(), b.ravel())])


@pytest.mark.parametrize("logn", [10, 12])
def test_polymul_vs_schoolbook(ntt, logn):
    N = 1 << logn
    moduli = P17[:3]
    log(f"case polymul N={N} vs schoolbook")
    a = si.poly_batch(5, 1, moduli, N)
    b = si.poly_batch(6, 1, moduli, N)
    plan = ntt.Plan(N, moduli)
    da, db = to_dev(a), to_dev(b)
    plan.forward(da)
    plan.forward(db)
    plan.pointwise(da, db, da)
    plan.inverse(da)
    got = from_dev(da).reshape(a.shape)
    for l, q in enumerate(moduli):
        np.testing.assert_array_equal(got[0, l], oracle.negacyclic_mul(a[0, l], b[0, l], q))


def test_polymul_full_size_two_ciphertexts(ntt):
    # N = 2^16, 24 limbs, 2 ciphertexts x 2 components: forward of all 4 polys
    # against the oracle in full; the negacyclic product against schoolbook
    # on a subset of limbs (sampled coefficients, O(N) each)
    w = si.workload_polymul_n16()
    log(f"case {w.name}")
    a = si.poly_batch(w.seed, 2, w.moduli, w.N)        # ciphertext A: 2 components
    b = si.poly_batch(w.seed + 1000, 2, w.moduli, w.N)  # ciphertext B
    plan = ntt.Plan(w.N, w.moduli)
    da, db = to_dev(a), to_dev(b)
    plan.forward(da)
    plan.forward(db)
    A = from_dev(da).reshape(a.shape)
    np.testing.assert_array_equal(A, oracle_fwd(a, w.moduli))
    np.testing.assert_array_equal(from_dev(db).reshape(b.shape), oracle_fwd(b, w.moduli))
    plan.pointwise(da, db, da)
    plan.inverse(da)
    c = from_dev(da).reshape(a.shape)
    rng = np.random.default_rng(0)
    for comp, l in ((0, 0), (1, 23), (0, 11)):
        q = w.moduli[l]
        for k in [0, 1, w.N - 1] + list(rng.integers(0, w.N, 4)):
            assert int(c[comp, l, k]) == oracle.negacyclic_coeff(a[comp, l], b[comp, l], q, int(k))


def test_sampled_direct_definition_full_size(ntt):
    # sampled outputs of the definition at the largest size
    N, moduli = 1 << 17, P18[:2]
    log("case sampled direct definition N=2^17")
    x = si.poly_batch(9, 1, moduli, N)
    plan = ntt.Plan(N, moduli)
    d = to_dev(x)
    plan.forward(d)
    X = from_dev(d).reshape(x.shape)
    for l, q in enumerate(moduli):
        for k in (0, 1, 12345, N - 1):
            assert int(X[0, l, k]) == oracle.ntt_direct_coeff(x[0, l], q, k)
        for j in (0, 7, N - 1):
            assert oracle.intt_direct_coeff(X[0, l], q, j) == int(x[0, l, j])


@pytest.mark.parametrize("logn", [5, 12, 16])
def test_edge_inputs(ntt, logn):
    N = 1 << logn
    moduli = P18[:2]
    log(f"case edge inputs N={N}")
    plan = ntt.Plan(N, moduli)
    cases = {
        "zeros": np.zeros((1, 2, N), np.uint64),
        "q-1": np.array([[[q - 1] * N for q in moduli]], np.uint64),
        "delta0": np.zeros((1, 2, N), np.uint64),
        "alternating": np.array([[[(q - 1) * (i & 1) for i in range(N)] for q in moduli]], np.uint64),
    }
    cases["delta0"][0, :, 0] = 1
    for name, x in cases.items():
        d = to_dev(x)
        plan.forward(d)
        X = from_dev(d).reshape(x.shape)
        np.testing.assert_array_equal(X, oracle_fwd(x, moduli), err_msg=name)
        if name == "delta0":
            assert (X == 1).all()
        plan.inverse(d)
        np.testing.assert_array_equal(from_dev(d).reshape(x.shape), x, err_msg=name)


def test_batch_one_limb_subset_and_ragged_batches(ntt):
    # batch sizes that leave partial workgroups (several polys per group)
    moduli = P18[:3]
    for N, batch in ((16, 5), (64, 7), (256, 3), (1024, 1)):
        run_roundtrip(ntt, N, moduli, batch=batch, seed=N + batch)


def test_repeatable(ntt):
    N, moduli = 1 << 16, P17[:4]
    log("case repeatability")
    x = si.poly_batch(2, 2, moduli, N)
    plan = ntt.Plan(N, moduli)
    outs = []
    for _ in range(3):
        d = to_dev(x)
        plan.forward(d)
        outs.append(from_dev(d))
    assert all((o == outs[0]).all() for o in outs)


def test_argument_errors_on_gpu(ntt):
    import torch
    plan = ntt.Plan(1024, P18[:1])
    lib = ntt.lib()
    t = torch.zeros(1024, dtype=torch.int64, device="cuda")
    assert lib.ntt_forward(plan.handle, t.data_ptr(), 0, None) == -1
    assert lib.ntt_forward(plan.handle, None, 1, None) == -1
    assert lib.ntt_forward(None, t.data_ptr(), 1, None) == -1
    assert lib.ntt_pointwise_mul(plan.handle, None, t.data_ptr(), t.data_ptr(), 1, None) == -1
    with pytest.raises(ntt.NttError):
        plan.set_variant(ntt.NTT_PATH_FOURSTEP, 5)
    with pytest.raises(ntt.NttError):
        plan.set_row_twist(4)


def test_stage_entry_points_compose(ntt):
    N, moduli = 1 << 16, P17[:3]
    log("case stage entry points")
    x = si.poly_batch(21, 2, moduli, N)
    plan = ntt.Plan(N, moduli)
    assert plan.variant[0] == ntt.NTT_PATH_FOURSTEP
    d = to_dev(x)
    plan.forward_stage(d, 0)
    plan.forward_stage(d, 1)
    np.testing.assert_array_equal(from_dev(d).reshape(x.shape), oracle_fwd(x, moduli))
    plan.inverse_stage(d, 0)
    plan.inverse_stage(d, 1)
    np.testing.assert_array_equal(from_dev(d).reshape(x.shape), x)
    small = ntt.Plan(1024, moduli)
    with pytest.raises(ntt.NttError):
        small.forward_stage(to_dev(si.poly_batch(1, 1, moduli, 1024)), 0)


@pytest.mark.parametrize("logn,bitrev,variant", [(16, False, None), (16, True, None), (15, False, None),
                                                  (12, False, None), (12, False, (3, 6)), (13, True, (3, 6)),
                                                  (16, False, (3, 7)), (15, True, (3, 9)), (17, False, None)])
@pytest.mark.parametrize("row_twist", [True, False])
def test_fused_pointwise_inverse(ntt, logn, bitrev, variant, row_twist):
    N, moduli = 1 << logn, P18[:3]
    log(f"case fused pointwise+inverse N={N} bitrev={bitrev} variant={variant} row_twist={row_twist}")
    plan = ntt.Plan(N, moduli, flags=ntt.NTT_ORDER_BITREV if bitrev else 0)
    if variant:
        plan.set_variant(*variant)
    plan.set_row_twist(row_twist)
    a = si.poly_batch(31, 2, moduli, N)
    b = si.poly_batch(32, 2, moduli, N)
    da, db = to_dev(a), to_dev(b)
    plan.forward(da)
    plan.forward(db)
    dc = to_dev(np.zeros_like(a))
    plan.pointwise_inverse(da, db, dc)
    got = from_dev(dc).reshape(a.shape)
    # reference: the unfused path, itself checked against the oracle elsewhere
    A = oracle_fwd(a, moduli)
    B = oracle_fwd(b, moduli)
    ref = oracle_inv(oracle.pointwise_batch(A, B, moduli)[0], moduli)
    np.testing.assert_array_equal(got, ref)
    plan.pointwise_inverse(da, db)          # aliasing: result into a
    np.testing.assert_array_equal(from_dev(da).reshape(a.shape), ref)
    if logn <= 12:
        for l, q in enumerate(moduli):
            np.testing.assert_array_equal(got[1, l], oracle.negacyclic_mul(a[1, l], b[1, l], q))


@pytest.mark.parametrize("logn,logn1,bitrev", [(14, 7, False), (16, 8, False), (17, 9, True)])
@pytest.mark.parametrize("row_twist", [True, False])
def test_fused_pointwise_inverse_u32(ntt, logn, logn1, bitrev, row_twist):
    """32-bit words: the fused product is a Montgomery product at 2^32 and the
    inverse column pass multiplies 2^32 back in; against the unfused oracle."""
    N, moduli = 1 << logn, Q32[:2]
    log(f"case fused pointwise+inverse u32 N={N} logn1={logn1} bitrev={bitrev} row_twist={row_twist}")
    plan = ntt.Plan(N, moduli, flags=ntt.NTT_WORD32 | (ntt.NTT_ORDER_BITREV if bitrev else 0))
    plan.set_variant(ntt.NTT_PATH_FOURSTEP, logn1)
    plan.set_row_twist(row_twist)
    a = si.poly_batch(51, 2, moduli, N)
    b = si.poly_batch(52, 2, moduli, N)
    da, db = to_dev(a, 32), to_dev(b, 32)
    plan.forward(da)
    plan.forward(db)
    dc = to_dev(np.zeros_like(a), 32)
    plan.pointwise_inverse(da, db, dc)
    ref = oracle_inv(oracle.pointwise_batch(oracle_fwd(a, moduli), oracle_fwd(b, moduli), moduli)[0], moduli)
    np.testing.assert_array_equal(from_dev(dc, 32).reshape(a.shape), ref)


@pytest.mark.parametrize("logn,logn1", [(14, 7), (16, 8), (17, 9)])
@pytest.mark.parametrize("row_twist", [True, False])
def test_fused_pointwise_inverse_exact_quotient(ntt, logn, logn1, row_twist):
    """The fused product + inverse with the exact Shoup quotient (lazy bound 2q)."""
    N, moduli = 1 << logn, P18[3:5]
    log(f"case fused pointwise+inverse exact N={N} logn1={logn1} row_twist={row_twist}")
    plan = ntt.Plan(N, moduli)
    plan.set_variant(ntt.NTT_PATH_FOURSTEP, logn1)
    plan.set_exact_quotient(True)
    plan.set_row_twist(row_twist)
    a = si.poly_batch(41, 2, moduli, N)
    b = si.poly_batch(42, 2, moduli, N)
    da, db = to_dev(a), to_dev(b)
    plan.forward(da)
    plan.forward(db)
    np.testing.assert_array_equal(from_dev(da).reshape(a.shape), oracle_fwd(a, moduli))
    plan.pointwise_inverse(da, db)
    A = oracle_fwd(a, moduli)
    B = oracle_fwd(b, moduli)
    ref = oracle_inv(oracle.pointwise_batch(A, B, moduli)[0], moduli)
    np.testing.assert_array_equal(from_dev(da).reshape(a.shape), ref)
    plan.close()
