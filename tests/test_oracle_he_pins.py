"""The oracle's HE steps pinned to the Chinese remainder theorem and to ring
algebra (see he_pins.py), at several basis sizes."""
import pytest

import he_pins


def test_tensor_identity():
    assert he_pins.check_tensor() == []


@pytest.mark.parametrize("N,moduli", [(1, (7681,)), (17, (998244353, 7681, 12289))])
def test_tensor_identity_shapes(N, moduli):
    assert he_pins.check_tensor(seed=11, N=N, moduli=moduli) == []


@pytest.mark.parametrize("L,K", [(3, 1), (2, 2), (5, 4), (8, 24), (24, 8)])
def test_base_conv_crt(L, K):
    assert he_pins.check_base_conv(seed=20 + L, N=24, L=L, K=K) == []


def test_base_conv_crt_one_source():
    # with one source prime alpha is always 0; only that special case applies
    f = he_pins.check_base_conv(seed=3, N=24, L=1, K=3)
    assert f == ["conv: alpha never varies"]


@pytest.mark.parametrize("L,K", [(1, 2), (3, 5), (8, 24)])
def test_mod_down_crt(L, K):
    assert he_pins.check_mod_down(seed=30 + L, N=20, L=L, K=K) == []


def test_crt_helper_against_definition():
    # Garner's reconstruction against a search over all values (tiny moduli)
    ms = [5, 7, 9 + 2]
    for X in range(5 * 7 * 11):
        assert he_pins.crt([X % m for m in ms], ms) == X


@pytest.mark.parametrize("L,K", [(3, 2), (9, 4)])
def test_conversions_with_61bit_primes(L, K):
    assert he_pins.check_base_conv(seed=40 + L, N=16, L=L, K=K, bits=61) == []
    assert he_pins.check_mod_down(seed=50 + L, N=16, L=L, K=K, bits=61) == []
