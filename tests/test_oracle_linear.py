"""Pins of the elementwise multiply with truncation (Alg. linear,
truncate-then-multiply, against multiply-then-truncate), test
infrastructure for the oracle's ``beaver_mul`` and ``mul_trunc``.

* The Beaver product reconstructs to x y mod 2^l for every share and
  triple (brute force at l = 4, random at l up to 64).
* Each truncation follows the exact SecureML form of Sec. 3 (e0 and e1
  terms from the shares; the form is brute-forced in
  test_oracle_truncation.py): Alg. linear gives T(x, floor(f/2)) T(y,
  ceil(f/2)), multiply-then-truncate gives T(x y, f).
* The e1 phenomenon of Sec. 4: after one multiplication of 31-bit values
  in Z_2^64 the product carries 62 bits and fails with probability
  |x y| / 2^64; truncating the factors first keeps every element intact.
"""

import numpy as np
import pytest

from oracle import philox, protocols as P, ring

from closed_forms import expected_trunc_prob

U = np.uint64
SEEDS = (0x0123456789ABCDEF, 0x0F0F0F0F12345678, 0x7777AAAA5555CCCC)


def _rand(rng, n, ell):
    v = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * U(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    return ring.red(v, ell)


def _signed(v, ell):
    return np.array([a - (1 << ell) if a >> (ell - 1) else a for a in np.asarray(v).tolist()], dtype=object)


def test_beaver_mul_brute_force_l4():
    """Every (x0, x1, y0, y1) in Z_16^4 with a random triple: x y mod 16."""
    ell = 4
    g = np.array(np.meshgrid(*[np.arange(16, dtype=U)] * 4, indexing="ij")).reshape(4, -1)
    rng = np.random.default_rng(4)
    n = g.shape[1]
    a0, b0, c0, a1, b1 = (_rand(rng, n, ell) for _ in range(5))
    z0, z1 = P.beaver_mul(g[0], g[1], g[2], g[3], ell, a0, b0, c0, a1, b1)
    x, y = ring.add(g[0], g[1], ell), ring.add(g[2], g[3], ell)
    assert np.array_equal(ring.add(z0, z1, ell), ring.mul(x, y, ell))


@pytest.mark.parametrize("ell", [1, 24, 32, 40, 64])
def test_beaver_mul_random_rings(ell):
    rng = np.random.default_rng(ell)
    n = 20000
    x0, x1, y0, y1, a0, b0, c0, a1, b1 = (_rand(rng, n, ell) for _ in range(9))
    z0, z1 = P.beaver_mul(x0, x1, y0, y1, ell, a0, b0, c0, a1, b1)
    x = [int(a) + int(b) for a, b in zip(x0.tolist(), x1.tolist())]
    y = [int(a) + int(b) for a, b in zip(y0.tolist(), y1.tolist())]
    want = np.array([(p * q) % (1 << ell) for p, q in zip(x, y)], dtype=U)
    assert np.array_equal(ring.add(z0, z1, ell), want)


@pytest.mark.parametrize("ell,f", [(8, 3), (8, 4), (16, 7), (64, 26), (64, 13)])
def test_truncate_then_multiply_exact_form(ell, f):
    """Alg. linear: the result is the product of the two SecureML
    truncations, each with its own e0 (and e1) from its shares."""
    rng = np.random.default_rng(ell * 100 + f)
    n = 4000 if ell > 8 else 65536
    x, y, Rx, Ry = (_rand(rng, n, ell) for _ in range(4))
    if ell == 8:
        x = np.repeat(np.arange(256, dtype=U), 256)
        y = np.tile(np.arange(256, dtype=U), 256)
    x0, x1 = ring.split(x, Rx, ell)
    y0, y1 = ring.split(y, Ry, ell)
    z0, z1 = P.mul_trunc(x0, x1, y0, y1, ell, f, P.TRUNC_BEFORE, SEEDS, 5)
    tx = expected_trunc_prob(x, Rx, ell, f // 2)
    ty = expected_trunc_prob(y, Ry, ell, f - f // 2)
    want = np.array([(a * b) % (1 << ell) for a, b in zip(tx.tolist(), ty.tolist())], dtype=object)
    assert np.array_equal(ring.add(z0, z1, ell).astype(object), want)


@pytest.mark.parametrize("ell,f", [(8, 3), (16, 7), (64, 26)])
def test_multiply_then_truncate_exact_form(ell, f):
    """Multiply-then-truncate: SecureML on the product's shares, whose offset
    is R' = -[xy]_1."""
    rng = np.random.default_rng(ell * 7 + f)
    n = 4000
    x0, x1, y0, y1 = (_rand(rng, n, ell) for _ in range(4))
    z0, z1 = P.mul_trunc(x0, x1, y0, y1, ell, f, P.TRUNC_AFTER, SEEDS, 6)
    a0, b0, c0, a1, b1 = philox.draw_beaver(SEEDS[1], SEEDS[2], 6, np.arange(n, dtype=U), ell, tag=philox.TAG_MUL)
    p0, p1 = P.beaver_mul(x0, x1, y0, y1, ell, a0, b0, c0, a1, b1)
    xy = ring.mul(ring.add(x0, x1, ell), ring.add(y0, y1, ell), ell)
    want = expected_trunc_prob(xy, ring.neg(p1, ell), ell, f)
    assert np.array_equal(ring.add(z0, z1, ell).astype(object), want)
    # f = 0: the plain product
    q0, q1 = P.mul_trunc(x0, x1, y0, y1, ell, 0, P.TRUNC_NONE, SEEDS, 6)
    assert np.array_equal(ring.add(q0, q1, ell), xy)


def _fixed(rng, n, lx, ell):
    v = rng.integers(-(1 << (lx - 1)) + 1, 1 << (lx - 1), size=n)
    return np.array([a % (1 << ell) for a in v.tolist()], dtype=U), v


def test_e1_of_one_multiplication():
    """Sec. 4's setting: l = 64, f = 26, 5 integer bits (|x|, |y| < 2^31).
    Multiply-then-truncate fails (off by about 2^(64-26)) with probability
    |x y| / 2^64 per element; at |x y| close to 2^62 that is 1/4.
    Truncate-then-multiply stays within a few units of x y / 2^26."""
    ell, f, n = 64, 26, 40000
    rng = np.random.default_rng(26)
    x = np.full(n, (1 << 31) - 1, dtype=U)
    y = np.full(n, (1 << 31) - 3, dtype=U)
    x0, x1 = ring.split(x, _rand(rng, n, ell), ell)
    y0, y1 = ring.split(y, _rand(rng, n, ell), ell)
    exact = (((1 << 31) - 1) * ((1 << 31) - 3)) >> f
    rate = ((1 << 31) - 1) * ((1 << 31) - 3) / 2.0 ** 64
    za = _signed(ring.add(*P.mul_trunc(x0, x1, y0, y1, ell, f, P.TRUNC_AFTER, SEEDS, 7), ell), ell)
    fails = np.array([abs(v - exact) > 1 for v in za.tolist()])
    sigma = np.sqrt(rate * (1 - rate) / n)
    assert abs(fails.mean() - rate) < 6 * sigma
    zb = _signed(ring.add(*P.mul_trunc(x0, x1, y0, y1, ell, f, P.TRUNC_BEFORE, SEEDS, 7), ell), ell)
    err = np.array([abs(v - exact) for v in zb.tolist()])
    assert err.max() < (1 << 19)           # about (|x| + |y|) / 2^13: the precision given up, no e1
    # random 31-bit factors: the failure rate is the mean of |x y| / 2^64
    xv, xs = _fixed(rng, n, 31, ell)
    yv, ys = _fixed(rng, n, 31, ell)
    x0, x1 = ring.split(xv, _rand(rng, n, ell), ell)
    y0, y1 = ring.split(yv, _rand(rng, n, ell), ell)
    za = _signed(ring.add(*P.mul_trunc(x0, x1, y0, y1, ell, f, P.TRUNC_AFTER, SEEDS, 8), ell), ell)
    prod = [int(a) * int(b) for a, b in zip(xs.tolist(), ys.tolist())]
    fails = np.array([abs(v - (p >> f)) > 1 for v, p in zip(za.tolist(), prod)])
    rate = float(np.mean([abs(p) for p in prod])) / 2.0 ** 64
    assert abs(fails.mean() - rate) < 6 * np.sqrt(rate / n)
    zb = _signed(ring.add(*P.mul_trunc(x0, x1, y0, y1, ell, f, P.TRUNC_BEFORE, SEEDS, 8), ell), ell)
    assert max(abs(v - (p >> f)) for v, p in zip(zb.tolist(), prod)) < (1 << 19)
