"""Pins of the oracle's truncation protocols (Alg. 1, Alg. 4, Alg. 5).

What fixes them, independently of the oracle's own code:
* the worked examples printed in Sec. 1 and Sec. 5.1 (tests/golden);
* exhaustive closed forms over every x and every mask R at l = 8, derived
  from Thm. (cut of a sum) and Cor. (SecureML failure) by splitting
  x + R' into its carry out of the low k bits (e0) and its wrap past 2^l;
* the exact SecureML failure count |x| per x (the paper's probability is
  the bound of Thm. 1, not an equality), the bound itself, and the fixed
  mask case of Sec. 4.1 that hides e1.
"""

import numpy as np
import pytest

from oracle import protocols as P
from oracle import ring

U = np.uint64


def _all_pairs(ell):
    x, R = np.meshgrid(np.arange(1 << ell, dtype=U), np.arange(1 << ell, dtype=U), indexing="ij")
    return x.ravel(), R.ravel()


def _floor_signed(x, ell, k):
    s = ring.signed(x, ell)
    return np.array([v >> k for v in s], dtype=object)   # Python >> floors


def test_worked_examples(golden):
    for name, alg, xb, Rb, k1, k2, expb, bits, *_ in golden("worked_examples.txt"):
        x, R, k1, k2, bits = int(xb, 2), int(Rb, 2), int(k1), int(k2), int(bits)
        x0, x1 = ring.split(np.array([x], U), np.array([R], U), 8)
        if alg == "prob":
            y0, y1 = P.trunc_prob(x0, x1, 8, k1)
        else:
            y0, y1 = P.trunc_det(x0, x1, 8, k1, k2)
        got = int(ring.add(y0, y1, bits)[0])
        assert got == int(expb, 2), name


def test_worked_example_shares():
    # Sec. 1: [x]_0 = 1111 0101, [x]_1 = 0101 0110 for x = 0100 1011, R = 1010 1010
    x0, x1 = ring.split(np.array([0b01001011], U), np.array([0b10101010], U), 8)
    assert int(x0[0]) == 0b11110101 and int(x1[0]) == 0b01010110


@pytest.mark.parametrize("k1,k2", [(k1, k2) for k1 in range(0, 8) for k2 in range(0, 8) if k1 + k2 < 8])
def test_trunc_det_closed_form_exhaustive(k1, k2):
    """For every x and R at l = 8: y0 + y1 = floor(sgn(x)/2^k1) + e0 mod 2^(l-k1-k2),
    e0 = [(x mod 2^k1) + (R mod 2^k1) >= 2^k1].  No e1, no domain restriction."""
    ell = 8
    m = ell - k1 - k2
    x, R = _all_pairs(ell)
    x0, x1 = ring.split(x, R, ell)
    y0, y1 = P.trunc_det(x0, x1, ell, k1, k2)
    got = ring.add(y0, y1, m)
    lowm = (1 << k1) - 1
    e0 = ((x.astype(object) & lowm) + (R.astype(object) & lowm)) >> k1
    exp = (_floor_signed(x, ell, k1) + e0) % (1 << m)
    assert np.array_equal(got.astype(object), exp)
    # output shares are canonical in the smaller ring
    assert int(y0.max()) < (1 << m) and int(y1.max()) < (1 << m)


@pytest.mark.parametrize("k", [1, 3, 4, 7])
def test_trunc_prob_closed_form_exhaustive(k):
    """SecureML at l = 8, every x, every R:
    y0 + y1 = floor(sgn(x)/2^k) + e0 + 2^(l-k) ([x < 0] - wrap) mod 2^l,
    wrap = [x + R >= 2^l] (x, R canonical).  e1 is the last term."""
    ell = 8
    x, R = _all_pairs(ell)
    x0, x1 = ring.split(x, R, ell)
    y0, y1 = P.trunc_prob(x0, x1, ell, k)
    got = ring.add(y0, y1, ell).astype(object)
    xo, Ro = x.astype(object), R.astype(object)
    lowm = (1 << k) - 1
    e0 = ((xo & lowm) + (Ro & lowm)) >> k
    wrap = (xo + Ro) >> ell
    neg = (xo >> (ell - 1)) & 1
    exp = (_floor_signed(x, ell, k) + e0 + (1 << (ell - k)) * (neg - wrap)) % (1 << ell)
    assert np.array_equal(got, exp)


def _failures_per_x(ell, k, R_values):
    """Count, per x, the masks R for which the SecureML output is off by more than e0."""
    xs = np.arange(1 << ell, dtype=U)
    fails = np.zeros(1 << ell, dtype=np.int64)
    for R in R_values:
        x0, x1 = ring.split(xs, np.full_like(xs, R), ell)
        y0, y1 = P.trunc_prob(x0, x1, ell, k)
        diff = (ring.add(y0, y1, ell).astype(object) - _floor_signed(xs, ell, k)) % (1 << ell)
        fails += np.array([d not in (0, 1) for d in diff], dtype=np.int64)
    return xs, fails


def test_trunc_prob_failure_count_is_abs_x():
    """Exhaustively at l = 8, k = 3: over all 256 masks, x fails for exactly |x| of them,
    i.e. P(e1 | x) = |x| / 2^l (Cor. of Sec. 3 made exact)."""
    ell, k = 8, 3
    xs, fails = _failures_per_x(ell, k, range(1 << ell))
    absx = np.abs(ring.signed(xs, ell).astype(np.int64))
    assert np.array_equal(fails, absx)


def test_trunc_prob_bound_of_theorem1():
    """Thm. 1: for x in the domain |x| < 2^l_x the failure probability is at most
    1 / 2^(l - l_x - 1).  Exhaustive at l = 10 for l_x = 4..7."""
    ell, k = 10, 2
    xs, fails = _failures_per_x(ell, k, range(1 << ell))
    absx = np.abs(ring.signed(xs, ell).astype(np.int64))
    for lx in range(4, 8):
        dom = absx < (1 << lx)
        worst = fails[dom].max() / (1 << ell)
        assert worst <= 1.0 / (1 << (ell - lx - 1))
        assert worst == ((1 << lx) - 1) / (1 << ell)


def test_fixed_mask_hides_e1():
    """Sec. 4.1: a fixed mask conceals e1.  With R' = 2^(l-1) (the SecureML analogue of
    the fixed r = 2^26), no x with |x| < 2^(l-1) ever fails; a random R exposes it."""
    ell, k = 8, 2
    xs, fails_fixed = _failures_per_x(ell, k, [1 << (ell - 1)])
    absx = np.abs(ring.signed(xs, ell).astype(np.int64))
    assert fails_fixed[absx < (1 << (ell - 1))].sum() == 0
    rng = np.random.default_rng(5)
    _, fails_rand = _failures_per_x(ell, k, rng.integers(0, 1 << ell, size=64))
    assert fails_rand[absx < (1 << (ell - 1))].sum() > 0


def test_trunc_prob_rate_large_ring():
    """l = 64 after one multiplication (l_x doubled to 62, Sec. 4.1): random masks fail
    at rate |x| / 2^64 per x.  Check the per-x rate within a binomial 5-sigma band."""
    ell, k = 64, 26
    rng = np.random.default_rng(11)
    for absx in (1 << 60, 1 << 61, 3 << 60):
        for sign in (1, -1):
            trials = 20000
            x = np.full(trials, (sign * absx) % (1 << 64), dtype=U)
            R = rng.integers(0, 1 << 63, size=trials, dtype=np.uint64) * U(2) + rng.integers(0, 2, size=trials, dtype=np.uint64)
            x0, x1 = ring.split(x, R, ell)
            y0, y1 = P.trunc_prob(x0, x1, ell, k)
            got = ring.add(y0, y1, ell).astype(object)
            fl = (sign * absx) >> k
            diff = [(int(g) - fl) % (1 << 64) for g in got]
            rate = np.mean([d not in (0, 1) for d in diff])
            q = absx / 2.0 ** 64
            assert abs(rate - q) <= 5 * np.sqrt(q * (1 - q) / trials) + 1e-9


def test_trunc_det_rejects_bad_k():
    x = np.zeros(2, U)
    with pytest.raises(ValueError):
        P.trunc_det(x, x, 8, 5, 3)
