"""Pins of the CPU oracle against things other than itself.

Each check names what fixes the expected value: the definition evaluated by
brute force, a library routine (sympy) on a special case, a closed form, or
an algebraic invariant. The paper prints no transform values, so no fixture
here comes from it.
"""
import numpy as np
import pytest
import sympy
from sympy.discrete.convolutions import convolution_ntt
from sympy.discrete.transforms import ntt as sympy_ntt

import oracle
import seeded_inputs as si

Q32 = si.Q_SMALL
P15 = si.ntt_primes(60, 15, 8)
P17 = si.ntt_primes(60, 17, 24)
P18 = si.ntt_primes(60, 18, 40)
SMALL_PRIMES = [Q32, 12289, 7681, P15[0], P17[0], P17[23], P18[0]]


def rand_vec(seed, q, N):
    return si.Stream(seed).uniform_mod(q, N)


# ---------------------------------------------------------------- scalars
@pytest.mark.parametrize("q", [Q32, P15[0], P17[5], P18[39]])
def test_scalar_ops_exact(q):
    vals = [0, 1, 2, q - 1, q - 2, q // 2, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, q // 3]
    vals = [v % q for v in vals]
    for a in vals:
        for b in vals:
            assert oracle.mulmod(a, b, q) == a * b % q
            assert int(oracle.lib().orc_addmod(a, b, q)) == (a + b) % q
            assert int(oracle.lib().orc_submod(a, b, q)) == (a - b) % q
    assert oracle.powmod(3, q - 1, q) == 1
    assert oracle.invmod(12345, q) * 12345 % q == 1


# ---------------------------------------------------------------- parameters
@pytest.mark.parametrize("q", SMALL_PRIMES + P17)
def test_qnr_and_root_against_sympy(q):
    c = oracle.smallest_qnr(q)
    # sympy's Legendre symbol: c is a non-residue, every 2 <= d < c is a residue
    assert sympy.legendre_symbol(c, q) == -1
    assert all(sympy.legendre_symbol(d, q) == 1 for d in range(2, c))
    for logn in (1, 3, 10, 12):
        N = 1 << logn
        if (q - 1) % (2 * N):
            continue
        r = oracle.psi(q, N)
        assert r == pow(c, (q - 1) // (2 * N), q)
        assert pow(r, N, q) == q - 1          # primitive 2N-th root: psi^N = -1
        assert pow(r, 2 * N, q) == 1
    # nested roots: psi_{N/2} = psi_N^2
    if (q - 1) % 1024 == 0:
        assert oracle.psi(q, 256) == pow(oracle.psi(q, 512), 2, q)


def test_root_convention_differs_from_primitive_root():
    # the reading of the paper's unnamed generator: smallest non-residue, not
    # the smallest primitive root; the two differ for this modulus
    q = P17[0]
    assert oracle.smallest_qnr(q) == 5
    assert sympy.primitive_root(q) == 10


def test_psi_rejects_unsupported_size():
    assert oracle.psi(Q32, 1 << 24) == 0   # 2^25 does not divide q-1


def test_prime_sets_are_prime_and_largest():
    for bits, s, lst in ((60, 15, P15), (60, 17, P17), (60, 18, P18)):
        step = 1 << s
        assert all(sympy.isprime(q) and q % step == 1 and q < 1 << bits for q in lst)
        assert lst == sorted(lst, reverse=True)
        # no prime of the form is skipped between 2^bits and the last one
        cand = ((1 << bits) - 1) // step * step + 1
        while cand >= lst[-1]:
            assert sympy.isprime(cand) == (cand in lst)
            cand -= step


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("q", SMALL_PRIMES)
@pytest.mark.parametrize("logn", range(1, 11))
def test_radix2_forward_equals_direct_definition(q, logn):
    N = 1 << logn
    if (q - 1) % (2 * N):
        pytest.skip("q does not support this N")
    x = rand_vec(logn * 7 + q % 1000, q, N)
    np.testing.assert_array_equal(oracle.ntt_forward(x, q), oracle.ntt_direct(x, q))


@pytest.mark.parametrize("logn", [3, 6, 8])
def test_direct_definition_against_sympy_ntt(logn):
    # special case reducing to a library routine: for q = 998244353 the
    # smallest non-residue 3 is also sympy's primitive root, so sympy's cyclic
    # NTT uses omega = 3^((q-1)/N) = psi^2, and the negacyclic transform is
    # that cyclic transform applied to the psi-twisted input.
    q, N = Q32, 1 << logn
    assert sympy.primitive_root(q) == oracle.smallest_qnr(q)
    x = rand_vec(99 + logn, q, N)
    r = oracle.psi(q, N)
    twisted = [int(v) * pow(r, j, q) % q for j, v in enumerate(x)]
    expect = [int(v) for v in sympy_ntt(twisted, q)]
    assert [int(v) for v in oracle.ntt_direct(x, q)] == expect
    assert [int(v) for v in oracle.ntt_forward(x, q)] == expect


@pytest.mark.parametrize("q", [Q32, P15[1], P17[0], P18[7]])
def test_closed_forms(q):
    N = 64
    r = oracle.psi(q, N)
    d0 = np.zeros(N, np.uint64); d0[0] = 1
    d1 = np.zeros(N, np.uint64); d1[1] = 1
    assert all(int(v) == 1 for v in oracle.ntt_forward(d0, q))               # NTT(1) = all ones
    assert [int(v) for v in oracle.ntt_forward(d1, q)] == [pow(r, 2 * k + 1, q) for k in range(N)]
    # x^j evaluates to psi^((2k+1) j)
    dj = np.zeros(N, np.uint64); dj[5] = 1
    assert [int(v) for v in oracle.ntt_forward(dj, q)] == [pow(r, (2 * k + 1) * 5, q) for k in range(N)]


@pytest.mark.parametrize("q", [Q32, P17[3]])
def test_linearity_and_shift(q):
    N = 256
    a, b = rand_vec(1, q, N), rand_vec(2, q, N)
    s = (a.astype(object) + b.astype(object)) % q
    A, B, S = oracle.ntt_forward(a, q), oracle.ntt_forward(b, q), oracle.ntt_forward(np.array(s, np.uint64), q)
    assert [int(v) for v in S] == [(int(x) + int(y)) % q for x, y in zip(A, B)]
    # multiplying by x is the negacyclic rotation z_0 = -a_{N-1}, z_k = a_{k-1};
    # in the NTT domain it multiplies X_k by psi^(2k+1)
    rot = np.array([(q - int(a[-1])) % q] + [int(v) for v in a[:-1]], np.uint64)
    r = oracle.psi(q, N)
    R = oracle.ntt_forward(rot, q)
    assert [int(v) for v in R] == [int(A[k]) * pow(r, 2 * k + 1, q) % q for k in range(N)]


@pytest.mark.parametrize("q", SMALL_PRIMES)
@pytest.mark.parametrize("logn", [1, 2, 5, 9, 12])
def test_round_trip(q, logn):
    N = 1 << logn
    if (q - 1) % (2 * N):
        pytest.skip("q does not support this N")
    x = rand_vec(logn + 5, q, N)
    np.testing.assert_array_equal(oracle.ntt_inverse(oracle.ntt_forward(x, q), q), x)


def test_round_trip_full_size_limb():
    q = P17[0]
    x = rand_vec(7, q, 1 << 16)
    np.testing.assert_array_equal(oracle.ntt_inverse(oracle.ntt_forward(x, q), q), x)


@pytest.mark.parametrize("q", [Q32, P15[0], P17[1]])
def test_inverse_direct_formula(q):
    N = 128
    X = rand_vec(17, q, N)
    inv = oracle.ntt_inverse(X, q)
    assert [oracle.intt_direct_coeff(X, q, j) for j in range(N)] == [int(v) for v in inv]
    # and the direct forward/inverse definitions are each other's inverse
    x = rand_vec(18, q, N)
    Xd = oracle.ntt_direct(x, q)
    assert [oracle.intt_direct_coeff(Xd, q, j) for j in range(N)] == [int(v) for v in x]


@pytest.mark.parametrize("q", [Q32, 12289, P15[2], P17[4]])
def test_schoolbook_against_sympy_linear_convolution(q):
    # library pin: sympy's NTT convolution gives the linear product; folding it
    # with x^N = -1 gives the negacyclic product
    N = 64
    a, b = rand_vec(3, q, N), rand_vec(4, q, N)
    lin = convolution_ntt([int(v) for v in a], [int(v) for v in b], prime=q if q != 12289 else 12289)
    lin = list(lin) + [0] * (2 * N - len(lin))
    expect = [(lin[k] - lin[k + N]) % q for k in range(N)]
    assert [int(v) for v in oracle.negacyclic_mul(a, b, q)] == expect


@pytest.mark.parametrize("q", [Q32] + P15[:2] + P17[:2])
@pytest.mark.parametrize("logn", [4, 10])
def test_convolution_theorem(q, logn):
    N = 1 << logn
    a, b = rand_vec(5 + logn, q, N), rand_vec(6 + logn, q, N)
    c = oracle.ntt_inverse(oracle.pointwise(oracle.ntt_forward(a, q), oracle.ntt_forward(b, q), q), q)
    np.testing.assert_array_equal(c, oracle.negacyclic_mul(a, b, q))


def test_convolution_theorem_full_size_sampled():
    q, N = P17[2], 1 << 16
    a, b = rand_vec(8, q, N), rand_vec(9, q, N)
    c = oracle.ntt_inverse(oracle.pointwise(oracle.ntt_forward(a, q), oracle.ntt_forward(b, q), q), q)
    for k in [0, 1, 2, 777, 32768, N - 2, N - 1]:
        assert int(c[k]) == oracle.negacyclic_coeff(a, b, q, k)


def test_direct_coeff_matches_full_direct():
    q, N = P18[0], 512
    x = rand_vec(10, q, N)
    X = oracle.ntt_direct(x, q)
    for k in [0, 1, 100, 511]:
        assert oracle.ntt_direct_coeff(x, q, k) == int(X[k])


def test_batched_drivers_match_single():
    moduli = P15[:3]
    x = si.poly_batch(11, 2, moduli, 256)
    y, used = oracle.ntt_forward_batch(x, moduli, nthreads=2)
    assert used == 2
    for b in range(2):
        for l, q in enumerate(moduli):
            np.testing.assert_array_equal(y[b, l], oracle.ntt_forward(x[b, l], q))
    z, _ = oracle.ntt_inverse_batch(y, moduli, nthreads=2)
    np.testing.assert_array_equal(z, x)
    p, _ = oracle.pointwise_batch(x, y, moduli)
    assert int(p[1, 2, 5]) == int(x[1, 2, 5]) * int(y[1, 2, 5]) % moduli[2]


def test_seeded_example_from_generator():
    # the generator's first draws and the transform of that vector, recomputed
    # from the definition (O(N^2)) rather than stored
    q, N = Q32, 1024
    x = si.Stream(1).uniform_mod(q, N)
    assert [int(v) for v in x[:4]] == [608340859, 800777064, 477127076, 477025590]
    np.testing.assert_array_equal(oracle.ntt_forward(x, q), oracle.ntt_direct(x, q))


# ---------------------------------------------------------------- cyclic (Eq. 3)
@pytest.mark.parametrize("logn", [1, 3, 6, 9])
def test_cyclic_against_sympy_ntt(logn):
    # library pin: sympy's ntt is the cyclic transform with omega = g^((q-1)/N),
    # g = sympy's primitive root = 3 = the smallest non-residue for this q
    q, N = Q32, 1 << logn
    x = rand_vec(200 + logn, q, N)
    expect = [int(v) for v in sympy_ntt([int(v) for v in x], q)]
    assert [int(v) for v in oracle.cyclic_forward(x, q)] == expect
    assert [oracle.cyclic_direct_coeff(x, q, k) for k in range(N)] == expect


@pytest.mark.parametrize("q", [Q32, P15[0], P17[2]])
def test_cyclic_closed_forms_and_round_trip(q):
    N = 128
    w = oracle.omega(q, N)
    assert pow(w, N, q) == 1 and pow(w, N // 2, q) == q - 1
    d1 = np.zeros(N, np.uint64); d1[1] = 1
    assert [int(v) for v in oracle.cyclic_forward(d1, q)] == [pow(w, k, q) for k in range(N)]
    ones = np.ones(N, np.uint64)
    X = oracle.cyclic_forward(ones, q)
    assert int(X[0]) == N % q and all(int(v) == 0 for v in X[1:])     # sum of all roots of unity
    x = rand_vec(300, q, N)
    np.testing.assert_array_equal(oracle.cyclic_inverse(oracle.cyclic_forward(x, q), q), x)
    # cyclic convolution theorem against the sympy linear product folded by x^N = 1
    a, b = rand_vec(301, q, N), rand_vec(302, q, N)
    lin = list(convolution_ntt([int(v) for v in a], [int(v) for v in b], prime=q)) + [0] * (2 * N)
    want = [(lin[k] + lin[k + N]) % q for k in range(N)]
    got = oracle.cyclic_inverse(oracle.pointwise(oracle.cyclic_forward(a, q), oracle.cyclic_forward(b, q), q), q)
    assert [int(v) for v in got] == want


@pytest.mark.parametrize("q", [Q32, P15[0], P18[3]])
@pytest.mark.parametrize("logn", [1, 2, 5, 8, 10])
def test_pease_and_stockham_equal_the_definition(q, logn):
    # brute force: the paper's constant-geometry (Pease) and autosort
    # (Stockham) orderings against the O(N^2) cyclic definition
    N = 1 << logn
    x = rand_vec(400 + logn, q, N)
    want = [oracle.cyclic_direct_coeff(x, q, k) for k in range(N)] if N <= 256 else \
        [int(v) for v in oracle.cyclic_forward(x, q)]
    assert [int(v) for v in oracle.pease_forward(x, q)] == want
    assert [int(v) for v in oracle.stockham_forward(x, q)] == want
