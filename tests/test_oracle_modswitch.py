"""Pins of the oracle's modulo switch (Alg. 6).

Sec. 5.3 states the property the protocol exists for: the output shares in
Z_p reconstruct to zero exactly when the input shares in Z_{2^l'} do.  The
correctness argument there also fixes the reconstructed value: s0 + s1 =
a0' + a1 - 2^l' (mod p) with a0' = a0, or 2^l' when a0 = 0.  Both are checked
for every pair of shares at small l' with every admissible prime.
"""

import numpy as np
import pytest
import sympy

from oracle import protocols as P
from oracle import params

U = np.uint64


def _primes_in(lo, hi):
    return [q for q in range(lo + 1, hi) if sympy.isprime(q)]


@pytest.mark.parametrize("ell", range(1, 10))
def test_zero_iff_zero_exhaustive(ell):
    a0, a1 = np.meshgrid(np.arange(1 << ell, dtype=U), np.arange(1 << ell, dtype=U), indexing="ij")
    a0, a1 = a0.ravel(), a1.ravel()
    for p in _primes_in(1 << ell, 1 << (ell + 1)):
        s0, s1 = P.mod_switch(a0, a1, ell, p)
        assert int(s0.max()) < p and int(s1.max()) < p
        zero_in = ((a0 + a1) % U(1 << ell)) == 0
        zero_out = ((s0 + s1) % U(p)) == 0
        assert np.array_equal(zero_in, zero_out), p
        # reconstructed value is v or v - 2^l' (mod p)
        v = ((a0 + a1) % U(1 << ell)).astype(object)
        rec = ((s0 + s1) % U(p)).astype(object)
        ok = (rec == v % p) | (rec == (v - (1 << ell)) % p)
        assert ok.all()


def test_worked_argument_cases():
    # the two cases of the Sec. 5.3 argument at l' = 4, p = 17 and p = 31
    for p in (17, 19, 23, 29, 31):
        s0, s1 = P.mod_switch(np.array([0], U), np.array([0], U), 4, p)
        assert (int(s0[0]), int(s1[0])) == (16 % p, (p - 16) % p)
        s0, s1 = P.mod_switch(np.array([5], U), np.array([11], U), 4, p)
        assert int(s0[0]) == 5 and (int(s0[0]) + int(s1[0])) % p == 0


def test_large_ring_random():
    rng = np.random.default_rng(3)
    for ell in (18, 31, 32):
        p = params.default_prime(ell)
        a0 = rng.integers(0, 1 << ell, size=4000, dtype=np.uint64)
        a1 = (U(1 << ell) - a0) % U(1 << ell)                  # zero
        a1[::2] = rng.integers(0, 1 << ell, size=2000, dtype=np.uint64)
        s0, s1 = P.mod_switch(a0, a1, ell, p)
        zin = ((a0 + a1) % U(1 << ell)) == 0
        zout = ((s0.astype(object) + s1.astype(object)) % p) == 0
        assert np.array_equal(zin, zout.astype(bool))
