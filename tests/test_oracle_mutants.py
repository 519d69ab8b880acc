"""Mutation test of the oracle's pins: builds of the oracle with one planted
mistake each (a dropped twist, psi instead of psi^-1, an off-by-one twiddle
index, a skipped stage, a missing N^-1, a swapped butterfly, a missing bit
reversal, a wrong sign in the definition or in the schoolbook wrap, a
transposed pointwise operand; in the HE steps: a dropped shat^-1 factor, a
dropped term, S in place of shat_i, a ModDown sign flip, a missing S^-1, a
wrong tensor operand) must each fail the battery of pins below,
which the real oracle passes. The pins compare against sympy, closed forms
and algebra, never against the oracle itself."""
import numpy as np
import pytest
import sympy
from sympy.discrete.convolutions import convolution_ntt
from sympy.discrete.transforms import ntt as sympy_ntt

import he_pins
import oracle
import seeded_inputs as si

Q = si.Q_SMALL
Q60 = si.ntt_primes(60, 17, 1)[0]
MUTANTS = {1: "dropped twist", 2: "psi^-1 twist", 3: "twiddle index +1", 4: "last stage skipped",
           5: "inverse without N^-1", 6: "definition with 2k-1", 7: "butterfly outputs swapped",
           8: "no bit reversal", 9: "schoolbook wrap added", 10: "pointwise a*a",
           11: "conversion without shat^-1", 12: "conversion drops the last term", 13: "S in place of shat_i",
           14: "ModDown sign flipped", 15: "ModDown without S^-1", 16: "tensor d1 with a1 b1"}


def battery():
    """Returns the list of pins that fail (empty when all hold)."""
    failed = []
    N = 64
    s = si.Stream(77)
    x, a, b = s.uniform_mod(Q, N), s.uniform_mod(Q, N), s.uniform_mod(Q, N)
    r = pow(3, (Q - 1) // (2 * N), Q)
    # sympy special case: negacyclic = cyclic (sympy) of the twisted input
    want = [int(v) for v in sympy_ntt([int(v) * pow(r, j, Q) % Q for j, v in enumerate(x)], Q)]
    if [int(v) for v in oracle.ntt_forward(x, Q)] != want:
        failed.append("forward vs sympy")
    if [int(v) for v in oracle.ntt_direct(x, Q)] != want:
        failed.append("definition vs sympy")
    d1 = np.zeros(N, np.uint64); d1[1] = 1
    if [int(v) for v in oracle.ntt_forward(d1, Q)] != [pow(r, 2 * k + 1, Q) for k in range(N)]:
        failed.append("NTT(x) closed form")
    if not np.array_equal(oracle.ntt_inverse(oracle.ntt_forward(x, Q), Q), x):
        failed.append("round trip")
    # inverse against its own definition would not catch a shared mistake; use
    # the known input instead: INTT(sympy spectrum) must return x
    if [int(v) for v in oracle.ntt_inverse(np.array(want, np.uint64), Q)] != [int(v) for v in x]:
        failed.append("inverse of sympy spectrum")
    lin = list(convolution_ntt([int(v) for v in a], [int(v) for v in b], prime=Q)) + [0] * (2 * N)
    neg = [(lin[k] - lin[k + N]) % Q for k in range(N)]
    if [int(v) for v in oracle.negacyclic_mul(a, b, Q)] != neg:
        failed.append("schoolbook vs sympy convolution")
    prod = oracle.ntt_inverse(oracle.pointwise(oracle.ntt_forward(a, Q), oracle.ntt_forward(b, Q), Q), Q)
    if [int(v) for v in prod] != neg:
        failed.append("convolution theorem vs sympy")
    return failed + he_pins.battery()


def test_real_oracle_passes_battery():
    oracle.use_library(None)
    assert battery() == []


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_planted_mistake_is_caught(k, tmp_path):
    path = oracle.build_variant(str(tmp_path / f"liboracle_mut{k}.so"), [f"ORC_MUTANT={k}"])
    oracle.use_library(path)
    try:
        failed = battery()
    finally:
        oracle.use_library(None)
    assert failed, f"mutant {k} ({MUTANTS[k]}) passed every pin"
