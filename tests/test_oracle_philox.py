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
import pytest

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


# ------------------------------------------------------------ the shuffle
# Pins of the digit-driven inside-out Fisher-Yates shuffle: the chunking rule
# against the product of the radices, each chunk's digits against the
# mixed-radix expansion of one big product floor(F M / 2^64) (Python
# integers, a different computation from the oracle's digit-by-digit
# extraction), the shuffle against brute force (a bijection onto all
# permutations) and hand-worked cases.

@pytest.mark.parametrize("n", range(2, 34))
def test_shuffle_chunks_follow_the_greedy_rule(n):
    import math
    chunks = philox.shuffle_chunks(n)
    radix = philox.shuffle_radices(n)
    assert radix == [2] + list(range(2, n + 1))
    assert [k for c in chunks for k in c] == list(range(n))       # in order, each digit once
    prods = [math.prod(radix[k] for k in c) for c in chunks]
    assert all(pr <= 1 << 32 for pr in prods)
    assert math.prod(prods) == 2 * math.factorial(n)
    for c, nxt in zip(chunks, chunks[1:]):                            # a chunk closes only when full
        assert math.prod(radix[k] for k in c) * radix[nxt[0]] > 1 << 32
    assert len(chunks) == (1 if n <= 12 else 2 if n <= 19 else 3 if n <= 26 else 4 if n <= 32 else 5)
    # the bias bound: the sum of M_c / 2^64 over the chunks
    assert sum(prods) / 2.0 ** 64 <= len(chunks) * 2.0 ** -32


def test_chunk_digits_extremes():
    radices = [2, 2, 3, 4, 5, 6, 7]
    zero = philox.chunk_digits(np.array([0], dtype=U), np.array([0], dtype=U), radices)
    assert [int(d[0]) for d in zero] == [0] * len(radices)
    top = philox.chunk_digits(np.array([0xFFFFFFFF], dtype=U), np.array([0xFFFFFFFF], dtype=U), radices)
    assert [int(d[0]) for d in top] == [m - 1 for m in radices]     # F = 2^64 - 1: every digit at its maximum
    half = philox.chunk_digits(np.array([0], dtype=U), np.array([1 << 31], dtype=U), [2, 2, 3])
    assert [int(d[0]) for d in half] == [1, 0, 0]                      # F = 1/2: t = 1, then F = 0


@pytest.mark.parametrize("n", [2, 3, 8, 12, 19, 20, 26, 33])
def test_shuffle_digits_are_one_mixed_radix_number_per_chunk(n):
    g = np.arange(7, 7 + 400, dtype=U) * U(2654435761)
    digits = philox.shuffle_digits(5, 9, g, n)
    radix = philox.shuffle_radices(n)
    for c, idx in enumerate(philox.shuffle_chunks(n)):
        blk = philox.block(5, 9, g, philox.TAG_SHUFFLE, c // 2)
        lo, hi = blk[2 * (c % 2)], blk[2 * (c % 2) + 1]
        M = 1
        for k in idx:
            M *= radix[k]
        for e in range(g.size):
            F = int(lo[e]) | int(hi[e]) << 32
            D = (F * M) >> 64                                          # one product, then its digits
            want = []
            for k in reversed(idx):
                D, d = divmod(D, radix[k])
                want.append(d)
            assert D == 0
            assert [int(digits[e, k]) for k in idx] == want[::-1], (n, c, e)


@pytest.mark.parametrize("n", range(1, 7))
def test_fisher_yates_is_a_bijection(n):
    import itertools
    import math
    tuples = list(itertools.product(*[range(i + 1) for i in range(n)]))   # j_0 = 0 (digit 0 is t), j_i in [0, i]
    perms = philox.fisher_yates(np.array(tuples, dtype=np.int64))
    assert len({tuple(p) for p in perms.tolist()}) == math.factorial(n) == len(tuples)
    assert np.all(np.sort(perms, axis=1) == np.arange(n))


def test_fisher_yates_worked_cases():
    # j = (t, 1, 0, 2): A = [0]; i=1, j=1: A[1] = 1; i=2, j=0: A[2] = A[0] = 0, A[0] = 2;
    # i=3, j=2: A[3] = A[2] = 0, A[2] = 3  ->  [2, 1, 3, 0]
    assert philox.fisher_yates(np.array([[1, 1, 0, 2]])).tolist() == [[2, 1, 3, 0]]
    for n in (2, 5, 19, 33):
        zero = philox.fisher_yates(np.zeros((1, n), dtype=np.int64))
        assert zero.tolist() == [[n - 1] + list(range(n - 1))]         # every j_i = 0: a rotation
        top = philox.fisher_yates(np.array([list(range(n))]))
        assert top.tolist() == [list(range(n))]                         # every j_i = i: the identity


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


def _tv(counts, m, total):
    """Statistical distance from uniform on m values of a map hit `counts`
    times per value out of `total` preimages: sum |c m - total| / (2 total m),
    the numerator summed exactly in integers."""
    num = int(np.abs(np.asarray(counts, dtype=np.int64) * m - total).sum())
    return num / (2 * total * m)


def test_stream_masks_only_where_the_layout_says():
    """N-bit fields of the mask stream for the default prime at N >= 17 only;
    an explicit prime, or N below 17, keeps the 32-bit words (64-bit words
    above 2^32).  Blocks per element: ceil(2 N^2 / 128) for the stream."""
    for lx in range(1, 33):
        n = lx + 1
        assert philox.stream_masks(n, default_prime(lx)) == (n >= 17), n
    assert not philox.stream_masks(19, 524269)                    # a prime below 2^19 - 1, not the default
    assert [philox.mask_blocks(n, default_prime(n - 1)) for n in (8, 16, 17, 19, 22, 32, 33)] == \
        [4, 8, 5, 6, 8, 16, 18]
    assert philox.mask_blocks(19, 524269) == 10 and philox.mask_blocks(33, 8589934487) == 33


def test_stream_mask_fields_read_as_bit_strings():
    """The fields R, Z of every slot, read from the stream as a string of
    characters (bit i of the stream at index i, the blocks in order), against
    draw_masks: pins the offsets N v, the fields that straddle words and
    blocks, and the clamp / mod."""
    g = np.array([0, 1, 77, (1 << 33) + 5, (1 << 47) + 123], dtype=U)
    for lx in (16, 17, 18, 19, 20, 21, 24, 27, 31, 32):
        n, p = lx + 1, default_prime(lx)
        r, z = philox.draw_masks(0x1234567890ABCDEF, 0x55, g, n, p)
        nb = -(-2 * n * n // 128)
        for e in range(g.size):
            bits = ""
            for b in range(nb):
                w = philox.block(0x1234567890ABCDEF, 0x55, g[e:e + 1], philox.TAG_MASK, b)
                bits += "".join(format(int(x[0]), "032b")[::-1] for x in w)   # bit i of the stream at index i
            for s in range(n):
                R = int(bits[2 * n * s:2 * n * s + n][::-1], 2)
                Z = int(bits[2 * n * s + n:2 * n * s + 2 * n][::-1], 2)
                assert int(r[e, s]) == min(max(R, 1), p - 1), (n, e, s)
                assert int(z[e, s]) == Z % p, (n, e, s)


def test_unpacked_masks_are_the_multiply_shift_of_words():
    """An explicit prime at N = 19 and the default prime at N = 16 keep the
    32-bit words of block s // 2 (computed here with Python integers)."""
    g = np.array([3, 99999], dtype=U)
    for n, p in ((19, 524269), (16, default_prime(15))):
        r, z = philox.draw_masks(7, 8, g, n, p)
        for e in range(g.size):
            for s in range(n):
                w = [int(x[0]) for x in philox.block(7, 8, g[e:e + 1], philox.TAG_MASK, s // 2)]
                R, Z = w[2 * (s % 2)], w[2 * (s % 2) + 1]
                assert int(r[e, s]) == 1 + (R * (p - 1) >> 32) and int(z[e, s]) == (Z * p) >> 32


def _field_tv(n, p):
    """Exact distance from uniform of r = clamp(R, 1, p - 1) and z = Z mod p
    over the 2^N field values R, Z: r has 1 taking 2 values, p - 1 taking
    c + 1 and the rest one; z has 0..c-1 taking 2 and the rest one."""
    c, tot = (1 << n) - p, 1 << n
    m = p - 1
    num_r = abs(2 * m - tot) + abs((c + 1) * m - tot) + (m - 2) * abs(m - tot)
    num_z = c * abs(2 * p - tot) + (p - c) * abs(p - tot)
    return num_r / (2 * tot * m), num_z / (2 * tot * p)


def test_stream_mask_bias_exhaustive():
    """Over every N-bit field value (N <= 21), the clamp and the reduction
    give the preimage counts the closed form assumes; the closed form then
    bounds the distance from uniform by 2^-15.4 at every N >= 17, within a
    factor 2 of the 32-bit multiply-shift's at N = 17..21 and far below it
    above."""
    def ms(m):                                      # the 32-bit multiply-shift: k values with q + 1 preimages
        k = (1 << 32) % m
        return 2 * k * (m - k) / (2 * (1 << 32) * m)
    for lx in (16, 17, 18, 19, 20):
        n, p = lx + 1, default_prime(lx)
        c = (1 << n) - p
        R = np.arange(1 << n, dtype=U)
        r = np.minimum(np.maximum(R, U(1)), U(p - 1))
        cr = np.bincount(r.astype(np.int64), minlength=p)
        assert cr[0] == 0 and cr[1] == 2 and cr[p - 1] == c + 1 and np.all(cr[2:p - 1] == 1)
        cz = np.bincount((R % U(p)).astype(np.int64), minlength=p)
        assert np.all(cz[:c] == 2) and np.all(cz[c:] == 1)
        assert (_tv(cr[1:], p - 1, 1 << n), _tv(cz, p, 1 << n)) == pytest.approx(_field_tv(n, p), rel=1e-12)
    for lx in range(16, 33):
        n, p = lx + 1, default_prime(lx)
        tv_r, tv_z = _field_tv(n, p)
        if n >= 17:
            assert tv_r <= 2 ** -15.4 and tv_z <= 2 ** -15.4, n
            assert tv_r <= 2 * ms(p - 1) and tv_z <= 2 * ms(p), n
        else:
            assert tv_r > 2 ** 6 * ms(p - 1)         # N = 17 is where N-bit fields stop costing bias


def test_stream_masks_in_range_and_uniform():
    N = 40000
    for lx in (16, 17, 18, 19, 20, 24, 32):
        p = default_prime(lx)
        r, z = philox.draw_masks(11, 12, np.arange(N, dtype=U), lx + 1, p)
        r, z = np.asarray(r, dtype=U), np.asarray(z, dtype=U)
        assert int(r.min()) >= 1 and int(r.max()) <= p - 1 and int(z.max()) <= p - 1
        # the top bits of r and z are uniform (bucketed by 2^(N - 6))
        sh = U(lx + 1 - 6)
        assert _chi2_ok(np.bincount((r.ravel() >> sh).astype(np.int64), minlength=64))
        assert _chi2_ok(np.bincount((z.ravel() >> sh).astype(np.int64), minlength=64))
        # neighbouring fields are independent: (r_0, z_2) top-bit pairs uniform
        pair = (r[:, 0] >> U(lx + 1 - 3)) * U(8) + (z[:, 2] >> U(lx + 1 - 3))
        assert _chi2_ok(np.bincount(pair.astype(np.int64), minlength=64))