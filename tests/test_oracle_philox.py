"""Properties of the oracle's Philox4x32-10 stream and draws.

The function itself is pinned against rocRAND's engine in
test_oracle_philox_rocrand.py (no published known-answer vector is
available in this environment); these tests pin what the definition and the
stream layout guarantee structurally and statistically: uniform, balanced
words, avalanche after ten rounds, disjoint
streams per (element, tag, block), valid permutations, draws in range and
uniform, and element-local randomness.
"""

import numpy as np

from oracle import philox
from oracle.params import default_prime

U = np.uint64


def _chi2_ok(counts, k=6.0):
    counts = np.asarray(counts, dtype=float)
    e = counts.sum() / counts.size
    chi2 = ((counts - e) ** 2 / e).sum()
    dof = counts.size - 1
    return abs(chi2 - dof) <= k * np.sqrt(2 * dof)


def test_words_uniform_and_balanced():
    g = np.arange(200000, dtype=U)
    w = np.concatenate(philox.block(0xDEADBEEFCAFEF00D, 42, g, philox.TAG_MASK, 3))
    for shift in (0, 8, 16, 24):
        assert _chi2_ok(np.bincount(((w >> U(shift)) & U(255)).astype(np.int64), minlength=256))
    bits = np.unpackbits(w.astype(np.uint32).view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.002


def test_avalanche():
    """Flipping one counter bit changes each output bit with probability ~1/2."""
    rng = np.random.default_rng(0)
    N = 20000
    c = [rng.integers(0, 1 << 32, size=N, dtype=np.uint64) for _ in range(4)]
    base = np.stack(philox.philox4x32_10(*c, 0x1234, 0x5678))
    for word in range(4):
        for bit in (0, 13, 31):
            c2 = [x.copy() for x in c]
            c2[word] ^= U(1 << bit)
            out = np.stack(philox.philox4x32_10(*c2, 0x1234, 0x5678))
            flips = np.unpackbits((out ^ base).astype(np.uint32).view(np.uint8)).mean()
            assert abs(flips - 0.5) < 0.01


def test_streams_disjoint():
    g = np.arange(5000, dtype=U)
    seen = set()
    for tag in (philox.TAG_SHUFFLE, philox.TAG_MASK, philox.TAG_RESP, philox.TAG_BEAVER):
        for b in range(3):
            words = philox.block(77, 5, g, tag, b)
            key = np.stack(words, axis=1)
            rows = {tuple(r) for r in key.tolist()}
            assert len(rows) == g.size
            assert not (rows & seen)
            seen |= rows
    # different seed or nonce -> different stream
    a = np.stack(philox.block(77, 5, g, 1, 0))
    assert not np.any(np.all(a == np.stack(philox.block(78, 5, g, 1, 0)), axis=0))
    assert not np.any(np.all(a == np.stack(philox.block(77, 6, g, 1, 0)), axis=0))


def test_high_element_index_bits_used():
    g = np.array([5, 5 + (1 << 32), 5 + (1 << 40)], dtype=U)
    b = np.stack(philox.block(1, 2, g, 1, 0), axis=1)
    assert len({tuple(r) for r in b.tolist()}) == 3


def test_shuffle_is_uniform_permutation():
    n = 8
    N = 80000
    t, sigma = philox.draw_shuffle(99, 1, np.arange(N, dtype=U), n)
    assert np.all(np.sort(sigma, axis=1) == np.arange(n))
    assert abs(t.astype(float).mean() - 0.5) < 0.01
    for slot in (0, 3, 7):
        assert _chi2_ok(np.bincount(sigma[:, slot], minlength=n))
    # pairs (sigma0, sigma1) uniform over the 56 ordered pairs
    assert _chi2_ok(np.bincount(sigma[:, 0] * n + sigma[:, 1], minlength=n * n)[
        [i * n + j for i in range(n) for j in range(n) if i != j]])
    # t independent of the first key's bits
    assert abs(np.mean(t[sigma[:, 0] == 0].astype(float)) - 0.5) < 0.03


def test_masks_in_range_and_uniform():
    N = 60000
    for lx in (7, 11, 18):
        p = default_prime(lx)
        r, z = philox.draw_masks(3, 4, np.arange(N, dtype=U), 4, p)
        assert int(r.min()) >= 1 and int(r.max()) <= p - 1
        assert int(z.max()) <= p - 1
        if p < 5000:
            assert _chi2_ok(np.bincount(r.ravel().astype(np.int64), minlength=p)[1:])
            assert _chi2_ok(np.bincount(z.ravel().astype(np.int64), minlength=p))
    p = default_prime(32)
    r, z = philox.draw_masks(3, 4, np.arange(2000, dtype=U), 3, p)
    assert min(r.ravel()) >= 1 and max(r.ravel()) <= p - 1 and max(z.ravel()) < p
    assert max(r.ravel()) > (1 << 32)                     # the 64-bit draw reaches the top


def test_rho_and_beaver_reduced():
    g = np.arange(1000, dtype=U)
    for ell in (24, 51, 64):
        rho = philox.draw_rho(1, 2, g, ell)
        assert int(rho.max()) < (1 << ell) if ell < 64 else True
        for v in philox.draw_beaver(1, 2, 3, g, ell):
            assert ell == 64 or int(v.max()) < (1 << ell)
