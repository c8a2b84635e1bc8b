"""Pins of the parties-apart DReLU oracle (Alg. 7 with each party's work on
its own, the round-1 messages bit-packed as they would cross a link).

* The packing is fixed by hand-computed examples and round trips for every
  window count, with the unused high bits zero.
* Every step before P2 is share-local: P0's messages do not change with
  [x]_1 (nor P1's with [x]_0), which is what lets drelu_send run on one
  share.
* send, reply and finish compose to the fused DReLU of the same seeds.
"""

import numpy as np
import pytest

from oracle import philox, protocols as P, ring
from oracle.params import default_prime

U = np.uint64
SEEDS = (0x1111222233334444, 0x5555666677778888, 0x99990000AAAABBBB)


def test_packing_worked_examples():
    # N = 2: slots (2, 1) -> bits 0-1 = 10b, bits 2-3 = 01b -> 0b0110
    assert P.pack_messages(np.array([[2, 1]], dtype=object), 2).tolist() == [[6]]
    # N = 3 (p = 7): slots (5, 0, 6) -> 101b at bit 0, 000b at bit 3, 110b at bit 6 -> 5 + 6 * 64
    assert P.pack_messages(np.array([[5, 0, 6]], dtype=object), 3).tolist() == [[389]]
    # N = 6: 36 bits, two words; slot 5 (value 63) straddles them: bits 30..35
    w = np.array([[0, 0, 0, 0, 0, 63]], dtype=object)
    assert P.pack_messages(w, 6).tolist() == [[3 << 30], [15]]


@pytest.mark.parametrize("npos", list(range(2, 34)))
def test_packing_round_trip(npos):
    rng = np.random.default_rng(npos)
    p = default_prime(npos - 1)
    n = 300
    w = np.array([[int(v) for v in rng.integers(0, p, size=npos)] for _ in range(n)], dtype=object)
    w[0, :] = p - 1
    words = P.pack_messages(w, npos)
    assert words.shape == (P.msg_words(npos), n)
    assert np.array_equal(P.unpack_messages(words, npos), w)
    spare = 32 * P.msg_words(npos) - npos * npos
    if spare:
        assert not np.any(words[-1].astype(object) >> (32 - spare))


def test_message_words_per_setting():
    assert [P.msg_words(n) for n in (8, 12, 19, 32, 33)] == [2, 5, 12, 32, 35]


@pytest.mark.parametrize("ell,lx,k_lo", [(64, 7, 11), (64, 18, 13), (64, 32, 0), (24, 7, 10)])
def test_messages_are_share_local(ell, lx, k_lo):
    rng = np.random.default_rng(lx)
    n = 2000
    p = default_prime(lx)
    x0, x1, x1b = (ring.red(rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * U(2), ell) for _ in range(3))
    g = np.arange(n, dtype=U)
    t, sigma = philox.draw_shuffle(SEEDS[0], 3, g, lx + 1)
    r, z = philox.draw_masks(SEEDS[0], 3, g, lx + 1, p)
    a0, a1 = P.drelu_round1(x0, x1, ell, lx, k_lo, p, t, sigma, r, z)
    b0, b1 = P.drelu_round1(x0, x1b, ell, lx, k_lo, p, t, sigma, r, z)
    c0, c1 = P.drelu_round1(x1, x1, ell, lx, k_lo, p, t, sigma, r, z)
    assert np.array_equal(a0, b0) and not np.array_equal(a1, b1)
    assert np.array_equal(a1, c1)


@pytest.mark.parametrize("ell,lx,k_lo", [(64, 7, 11), (64, 18, 13), (64, 31, 0), (64, 32, 0), (32, 8, 8), (8, 3, 1)])
def test_split_equals_fused(ell, lx, k_lo):
    rng = np.random.default_rng(ell + lx)
    n = 3000
    p = default_prime(lx)
    x = ring.red(rng.integers(-(1 << (k_lo + lx - 2)), 1 << (k_lo + lx - 2), size=n).astype(np.int64).view(U), ell)
    x0, x1 = ring.split(x, ring.red(rng.integers(0, 1 << 63, size=n, dtype=np.uint64), ell), ell)
    m0 = P.drelu_send(0, x0, ell, lx, k_lo, p, SEEDS, 5, elem_base=77)
    m1 = P.drelu_send(1, x1, ell, lx, k_lo, p, SEEDS, 5, elem_base=77)
    d0, d1 = P.drelu_reply(m0, m1, ell, lx, p, SEEDS, 5, elem_base=77)
    y0 = P.drelu_finish(0, d0, ell, lx, SEEDS, 5, elem_base=77)
    y1 = P.drelu_finish(1, d1, ell, lx, SEEDS, 5, elem_base=77)
    e0, e1, w0, w1 = P.drelu(x0, x1, ell, lx, k_lo, p, SEEDS, 5, elem_base=77)
    assert np.array_equal(y0, e0) and np.array_equal(y1, e1)
    assert np.array_equal(P.unpack_messages(m0, lx + 1), np.asarray(w0, dtype=object))
    assert np.array_equal(P.unpack_messages(m1, lx + 1), np.asarray(w1, dtype=object))
