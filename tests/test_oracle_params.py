"""Pins of the oracle's parameter logic against a library routine (sympy)."""

import numpy as np
import pytest
import sympy

from oracle import params


@pytest.mark.parametrize("lx", range(1, 33))
def test_default_prime_is_largest_below(lx):
    p = params.default_prime(lx)
    assert p == sympy.prevprime(1 << (lx + 1))
    assert (1 << lx) < p < (1 << (lx + 1))
    assert p.bit_length() == lx + 1          # notation table: bit length l_x + 1


def test_named_primes():
    # textbook values: Mersenne 2^19 - 1, 2^32 - 5, 2^33 - 9, and the small ones of the configs
    assert params.default_prime(18) == (1 << 19) - 1
    assert params.default_prime(31) == (1 << 32) - 5
    assert params.default_prime(32) == (1 << 33) - 9
    assert params.default_prime(7) == 251
    assert params.default_prime(8) == 509
    assert params.default_prime(11) == 4093


def test_is_prime_matches_sympy():
    rng = np.random.default_rng(0)
    for n in list(range(0, 3000)) + [int(v) for v in rng.integers(1, 1 << 62, size=3000, dtype=np.int64)]:
        assert params.is_prime(n) == sympy.isprime(n)
    for n in (2**61 - 1, 2**31 - 1, 561, 1105, 3215031751):   # primes and Carmichael/strong pseudoprimes
        assert params.is_prime(n) == sympy.isprime(n)


def test_check_drelu():
    params.check_drelu(64, 18, 13, (1 << 19) - 1)
    params.check_drelu(64, 32, 0, (1 << 33) - 9)
    params.check_drelu(51, 11, 13, 4093)
    params.check_drelu(24, 7, 10, 251)
    assert not sympy.isprime(524285)
    for bad in [(64, 18, 29, (1 << 19) - 1),      # k_lo + 2 l_x > l
                (64, 18, 13, (1 << 19) + 1),      # p above the range
                (64, 18, 13, 524285),             # in range, composite (5 * 104857)
                (65, 7, 0, 251), (64, 7, 0, 257)]:
        with pytest.raises(ValueError):
            params.check_drelu(*bad)


def test_keybit_window():
    # Tab. 5 combinations at f = 13: 5 + 2 keeps 2 fractional bits -> drop 11 low bits
    assert params.keybit_window(13, 5, 2) == (11, 7)
    assert params.keybit_window(13, 7, 0) == (13, 7)
    assert params.keybit_window(13, 17, 1) == (12, 18)
    assert params.guard_bound(13, 18) == 1 << 30
