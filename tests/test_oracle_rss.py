"""Pins of the replicated-sharing (RSS) DReLU / ReLU oracle (Alg. drelu2 and
the RSS ReLU of the appendix).

* The replicated-sharing product is checked by brute force on a small ring:
  every share triple of u and v reconstructs to u v.
* The preprocessing's sharings reconstruct to what they share: [t] to t, [s]
  to the bit s, [s xor t] to s xor t, and each zero sharing to 0.
* The output reconstructs to the closed form of the DReLU (derived from the
  appendix's lemmas, brute-forced in test_oracle_drelu.py) for the 2-of-2
  input ([x]_0 + [x]_1, [x]_2): R' = -[x]_2.  With key bits the band follows
  the carry c'_0 of that offset, which pins P0's input as [x]_0 + [x]_1.
* The ReLU output reconstructs to x DReLU(x) exactly.
* P2's public reply D'' is a fair coin whatever x is (s hides D').
"""

import numpy as np
import pytest

from oracle import philox, protocols as P, ring
from oracle.params import default_prime

from closed_forms import expected_dprime, in_exact_domain

U = np.uint64
SEEDS5 = (0x0123_4567_89AB_CDEF, 0x1357_9BDF_0246_8ACE, 0x0F1E_2D3C_4B5A_6978, 0x7766_5544_3322_1100,
          0x5A5A_A5A5_3C3C_C3C3)


def _rand(rng, N, ell):
    return ring.red(rng.integers(0, 1 << 63, size=N, dtype=np.uint64) * U(2) + rng.integers(0, 2, size=N,
                                                                                         dtype=np.uint64), ell)


def _rss_share(x, rng, ell):
    """x -> ([x]_0, [x]_1, [x]_2) with [x]_0, [x]_1 uniform."""
    a, b = _rand(rng, x.size, ell), _rand(rng, x.size, ell)
    return [a, b, ring.sub(ring.sub(x, a, ell), b, ell)]


def test_rss_mul_brute_force_l3():
    """Every share triple of u and every share triple of v in Z_8, with a
    random zero sharing: z reconstructs to u v mod 8."""
    ell = 3
    g = np.array(np.meshgrid(*[np.arange(8, dtype=U)] * 6, indexing="ij")).reshape(6, -1)
    u, v = [g[0], g[1], g[2]], [g[3], g[4], g[5]]
    rng = np.random.default_rng(1)
    gamma = P.zero_sharing([_rand(rng, g.shape[1], ell) for _ in range(3)], ell)
    z = P.rss_mul(u, v, gamma, ell)
    want = ring.mul(P.rss_reconstruct(u, ell), P.rss_reconstruct(v, ell), ell)
    assert np.array_equal(P.rss_reconstruct(z, ell), want)


@pytest.mark.parametrize("ell", [1, 8, 24, 32, 51, 64])
def test_rss_mul_random_rings(ell):
    rng = np.random.default_rng(ell)
    N = 20000
    u, v = [_rand(rng, N, ell) for _ in range(3)], [_rand(rng, N, ell) for _ in range(3)]
    gamma = P.zero_sharing([_rand(rng, N, ell) for _ in range(3)], ell)
    z = P.rss_mul(u, v, gamma, ell)
    uu, vv = P.rss_reconstruct(u, ell), P.rss_reconstruct(v, ell)
    want = np.array([(a * b) % (1 << ell) for a, b in zip(uu.tolist(), vv.tolist())], dtype=U)
    assert np.array_equal(P.rss_reconstruct(z, ell), want)


@pytest.mark.parametrize("ell", [1, 24, 64])
def test_preprocessing_sharings_reconstruct(ell):
    N = 50000
    g = np.arange(N, dtype=U)
    t, _ = philox.draw_shuffle(SEEDS5[0], 77, g, 8)
    d = philox.draw_rss(SEEDS5[3], SEEDS5[2], SEEDS5[4], 77, g, ell, relu=True)
    ts, ss, sxt = P.rss_preprocess(t, d, ell)
    assert np.array_equal(P.rss_reconstruct(ts, ell), t)
    assert np.array_equal(P.rss_reconstruct(ss, ell), d["s"])
    assert np.array_equal(P.rss_reconstruct(sxt, ell), d["s"] ^ t)
    for key in ("alpha", "alpha_st", "alpha_relu"):
        assert not np.any(P.rss_reconstruct(P.zero_sharing(d[key], ell), ell))
    # s and t are fair, independent coins
    for bits in (t, d["s"], d["s"] ^ t):
        assert abs(float(bits.mean()) - 0.5) < 6 * 0.5 / np.sqrt(N)
    if ell == 64:
        # every share of [t] and [s] is spread over the whole ring (top bit fair)
        for sh in ts + ss:
            assert abs(float((sh >> U(63)).mean()) - 0.5) < 6 * 0.5 / np.sqrt(N)


SETTINGS = [(8, 3, 0), (8, 3, 2), (12, 4, 2), (16, 6, 4), (64, 7, 11), (64, 18, 13), (64, 31, 0), (64, 32, 0),
            (51, 11, 13), (24, 7, 10), (32, 8, 8)]


@pytest.mark.parametrize("ell,lx,k_lo", SETTINGS)
def test_rss_drelu_relu_closed_form(ell, lx, k_lo):
    """Random x inside the guard domain (and the key-bit band, and 0): the
    DReLU reconstructs to D' xor t with D' of the closed form for the 2-of-2
    input ([x]_0 + [x]_1, [x]_2), the ReLU to x DReLU(x)."""
    p = default_prime(lx)
    rng = np.random.default_rng(ell * 1000 + lx * 10 + k_lo)
    N = 3000
    bound = 1 << (k_lo + lx - 1)
    xs = rng.integers(-bound + 1, bound, size=N)
    xs[:60] = rng.integers(-(1 << k_lo), (1 << k_lo) + 1, size=60)
    xs[60] = 0
    x = np.array([v % (1 << ell) for v in xs.tolist()], dtype=U)
    sh = _rss_share(x, rng, ell)
    nonce = 0xC0FFEE + lx
    y, w0, w1 = P.rss_drelu(*sh, ell, lx, k_lo, p, SEEDS5, nonce)
    g = np.arange(N, dtype=U)
    t, _ = philox.draw_shuffle(SEEDS5[0], nonce, g, lx + 1)
    Rp = ring.neg(sh[2], ell)                            # [x]_0 + [x]_1 = x + R'
    dr = P.rss_reconstruct(y, ell)
    assert np.array_equal(dr, expected_dprime(x, Rp, t, ell, k_lo) ^ t)
    outside = np.abs(xs) >= (1 << k_lo)
    assert np.array_equal(dr[outside], (xs[outside] > 0).astype(U))
    if k_lo == 0:
        assert int(dr[60]) == int(t[60])
    # round 1 is Alg. 7's, on the 2-of-2 input
    _, _, v0, v1 = P.drelu(ring.add(sh[0], sh[1], ell), sh[2], ell, lx, k_lo, p, SEEDS5[:3], nonce)
    assert np.array_equal(w0, v0) and np.array_equal(w1, v1)
    # ReLU: same round 1 and the same DReLU bit, times x at full precision
    yr, u0, u1 = P.rss_relu(*sh, ell, lx, k_lo, p, SEEDS5, nonce)
    assert np.array_equal(u0, w0) and np.array_equal(u1, w1)
    assert np.array_equal(P.rss_reconstruct(yr, ell), ring.mul(x, dr, ell))
    dom = in_exact_domain(x, t, ell, lx, k_lo)
    assert dom[outside].all()


def test_rss_drelu_exhaustive_l8():
    """Every x in Z_256 under several share splits: the closed form holds on
    the exact domain, and the ReLU identity for every x."""
    ell, lx, k_lo = 8, 3, 1
    p = default_prime(lx)
    rng = np.random.default_rng(8)
    x = np.tile(np.arange(256, dtype=U), 40)
    sh = _rss_share(x, rng, ell)
    g = np.arange(x.size, dtype=U)
    y, _, _ = P.rss_drelu(*sh, ell, lx, k_lo, p, SEEDS5, 5)
    t, _ = philox.draw_shuffle(SEEDS5[0], 5, g, lx + 1)
    dr = P.rss_reconstruct(y, ell)
    dom = in_exact_domain(x, t, ell, lx, k_lo)
    assert dom.sum() > 0.05 * x.size                 # about 23 of the 256 values
    assert np.array_equal(dr[dom], (expected_dprime(x, ring.neg(sh[2], ell), t, ell, k_lo) ^ t)[dom])
    assert np.all((dr == 0) | (dr == 1))
    yr, _, _ = P.rss_relu(*sh, ell, lx, k_lo, p, SEEDS5, 5)
    assert np.array_equal(P.rss_reconstruct(yr, ell), ring.mul(x, dr, ell))


def test_p2_reply_is_a_fair_coin():
    """For x all positive (D' = 1 - t everywhere) P2's public bit D'' = s xor D'
    is still a fair coin, and independent of t."""
    ell, lx, k_lo = 64, 7, 11
    p = default_prime(lx)
    N = 40000
    rng = np.random.default_rng(3)
    x = np.full(N, 12345 << 11, dtype=U)
    sh = _rss_share(x, rng, ell)
    g = np.arange(N, dtype=U)
    d = philox.draw_rss(SEEDS5[3], SEEDS5[2], SEEDS5[4], 9, g, ell, relu=False)
    _, w0, w1 = P.rss_drelu(*sh, ell, lx, k_lo, p, SEEDS5, 9)
    dpp = P.p2_zero_test(w0, w1, p) ^ d["s"]
    t, _ = philox.draw_shuffle(SEEDS5[0], 9, g, lx + 1)
    sig = 6 * 0.5 / np.sqrt(N)
    assert abs(float(dpp.mean()) - 0.5) < sig
    assert abs(float(dpp[t == 0].mean()) - 0.5) < 2 * sig and abs(float(dpp[t == 1].mean()) - 0.5) < 2 * sig


def test_rss_randomness_is_element_local():
    """Element g gets the same output alone, at another position, or with
    elem_base: every draw is indexed by the global element index."""
    ell, lx, k_lo = 64, 18, 13
    p = default_prime(lx)
    rng = np.random.default_rng(4)
    x = ring.red(rng.integers(-(1 << 29), 1 << 29, size=64).astype(np.int64).view(U), ell)
    sh = _rss_share(x, rng, ell)
    y, _, _ = P.rss_relu(*sh, ell, lx, k_lo, p, SEEDS5, 11, elem_base=1000)
    idx = np.array([5, 17, 63])
    ys, _, _ = P.rss_relu(*[s[idx] for s in sh], ell, lx, k_lo, p, SEEDS5, 11, g=(idx + 1000).astype(U))
    for j in range(3):
        assert np.array_equal(ys[j], y[j][idx])


def test_rss_msg_bits():
    """Link counts at Tab. 1's key-bit setting (l = 64, l_x = 7, p = 251):
    round 1 carries (l_x + 1)^2 = 64 bits per share-holder, as in Alg. 7."""
    bits, rounds = P.msg_bits("rss_drelu", 64, 7, 251)
    assert bits == [64 + 64, 64, 128, 128, 0, 64] and rounds == 2
    bits, rounds = P.msg_bits("rss_relu", 64, 7, 251)
    assert bits == [64 + 128, 64, 128, 192, 0, 128] and rounds == 3
    # the product adds one reshare on each link P_j -> P_{j-1}
    d, _ = P.msg_bits("rss_drelu", 64, 18, 524287)
    r, _ = P.msg_bits("rss_relu", 64, 18, 524287)
    assert [b - a for a, b in zip(d, r)] == [64, 0, 0, 64, 0, 64]


def test_each_secret_bit_sits_on_the_share_its_outsider_lacks():
    """P2 knows seed_012, hence every alpha, so t must sit on the one share of
    [t] that P2 does not hold ([t]_1; P2 holds shares 2 and 0).  P1 knows
    seed_012 and seed_12, hence [s]_1 and [s]_2, so s must enter only [s]_0
    (P1 holds shares 1 and 2).  Flipping t or s changes exactly that share."""
    ell, N = 64, 1000
    g = np.arange(N, dtype=U)
    t, _ = philox.draw_shuffle(SEEDS5[0], 3, g, 8)
    d = philox.draw_rss(SEEDS5[3], SEEDS5[2], SEEDS5[4], 3, g, ell, relu=False)
    ts, ss, _ = P.rss_preprocess(t, d, ell)
    ts2, ss2, _ = P.rss_preprocess(t ^ U(1), d, ell)
    assert np.array_equal(ts[0], ts2[0]) and np.array_equal(ts[2], ts2[2])
    assert not np.any(ts[1] == ts2[1])
    d2 = dict(d, s=d["s"] ^ U(1))
    _, ss3, _ = P.rss_preprocess(t, d2, ell)
    assert np.array_equal(ss[1], ss3[1]) and np.array_equal(ss[2], ss3[2])
    assert not np.any(ss[0] == ss3[0])
