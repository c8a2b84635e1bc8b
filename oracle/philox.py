"""Philox4x32-10 and the protocol's random draws (test infrastructure only).

The paper states only that P0 and P1 derive the flip, the shuffle and the
masks from seed_01 (Alg. 7), that P2 answers with a fresh sharing of its bit,
and that the Beaver triple comes from seed_02 / seed_12 (Alg. 8,
preprocessing).  It fixes no
generator.  This module is the build's definition, written from the
published description of Philox4x32 (Salmon, Moraes, Dror, Shaw, "Parallel
Random Numbers: As Easy as 1, 2, 3", SC'11):

* state: four 32-bit counter words (c0, c1, c2, c3), key (k0, k1);
* one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 64-bit
  products), new state = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
* ten rounds; before every round after the first the key is bumped by the
  Weyl constants (k0 += W0, k1 += W1 mod 2^32).

Counter layout, for element index g (< 2^48), a tag, and a block index b:
  c0 = g mod 2^32,  c1 = (g >> 32) | tag << 16 | b << 24,
  c2 = nonce mod 2^32,  c3 = nonce >> 32,   key = (seed mod 2^32, seed >> 32).
Every draw is therefore a pure function of (seed, nonce, g, tag, b): the same
element gets the same randomness alone, in a batch, or under any schedule.

Draws (no rejection; multiply-shift, whose statistical distance from
uniform is k (m - k) / (m 2^B) for m values drawn from B bits, k = 2^B mod m,
or N-bit fields, below):
  TAG_SHUFFLE (seed_01): the flip t and the permutation sigma of the N
    window positions come from N digits: digit 0 is t (radix 2), digit i
    (1 <= i < N) is j_i in [0, i] (radix i + 1), the choices of an
    inside-out Fisher-Yates shuffle: A[0] = 0, then for i = 1..N-1
    A[i] = A[j_i], A[j_i] = i; slot s of the shuffled array receives window
    position sigma(s) = A[s].  The digits are cut from 64-bit chunks
    F_c = w_{2c} | w_{2c+1} << 32 of the stream (word i is word i % 4 of
    block i // 4): digits go to chunk 0 in order while the product M_c of
    the chunk's radices stays <= 2^32, then to chunk 1, and so on.  Within a
    chunk, digit d of radix m is floor(F m / 2^64) and F becomes F m mod
    2^64, so the chunk's digits are the mixed-radix digits of
    floor(F_c M_c / 2^64), whose distance from uniform on [0, M_c) is at
    most M_c / 2^64 <= 2^-32.  The shuffle is a bijection from the digit
    tuples onto (t, sigma), so (t, sigma) is within (number of chunks) *
    2^-32 of uniform: two chunks (one block) at N <= 19, five at N = 33.
  TAG_MASK (seed_01), p < 2^32: block s//2 words 2(s%2), 2(s%2)+1 are
    (R, Z) of slot s;  r_s = 1 + floor(R (p-1) / 2^32) in Z_p^*,
    z_s = floor(Z p / 2^32) in Z_p.   p > 2^32: block s gives 64-bit
    R = w0 | w1 << 32, Z = w2 | w3 << 32 and the same formulas over 2^64.
  TAG_MASK, as a bit stream (``stream_masks``: the default prime
    p = 2^N - c of N = l_x + 1 >= 17 bits): the stream's bits are numbered
    0, 1, ... (bit i is bit i % 32 of word i // 32, word w is word w % 4 of
    block w // 4), and value v = 2s (R of slot s) or 2s + 1 (Z of slot s)
    is the N-bit field at bits [N v, N v + N); r_s = min(max(R, 1), p - 1)
    in Z_p^*, z_s = Z mod p.  The distance from uniform is (c + 1) / 2^N for
    r and about c / 2^N for z, at most 2^-15.4 (N = 18) and 2^-18 at
    N = 19, within a factor 2 of the 32-bit multiply-shift's at N = 17..21;
    an element's 2N fields take ceil(2 N^2 / 128) blocks (6 at N = 19, 18 at
    N = 33), where 32- or 64-bit words per value would take ceil(N / 2) or
    N.
  TAG_RESP (seed_02): rho = (w0 | w1 << 32) mod 2^l of block 0.
  TAG_BEAVER: seed_02 block 0 -> [a]_0 = w0|w1<<32, [b]_0 = w2|w3<<32;
    seed_02 block 1 -> [c]_0 = w0|w1<<32;  seed_12 block 0 -> [a]_1, [b]_1.
  TAG_RSS (replicated sharing, Alg. drelu2 in the appendix): the 64-bit
    values V_k = w_{2k} | w_{2k+1} << 32 of the seed_012 stream (word 2k of
    the stream is word 2k % 4 of block 2k // 4), each reduced mod 2^l:
      V_0, V_1, V_2 = alpha_0, alpha_1, alpha_2 (the sharing of t),
      V_3 = [s]_1,
      V_4, V_5, V_6 = alpha'_0..2 (zero sharing of the product [s][t]),
      V_7, V_8, V_9 = alpha''_0..2 (zero sharing of the ReLU product);
    seed_12 block 0: [s]_2 = w0 | w1 << 32;  seed_2 block 0: s = w0 & 1.
  TAG_MUL (the Beaver triple of an elementwise product, Alg. linear): the
    layout of TAG_BEAVER under its own tag.
"""

import numpy as np

from .params import default_prime
from .ring import U64, red

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85

TAG_SHUFFLE = 1
TAG_MASK = 2
TAG_RESP = 3
TAG_BEAVER = 4
TAG_RSS = 5
TAG_MUL = 6

_M32 = U64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, key0: int, key1: int):
    """Ten Philox4x32 rounds on uint64 arrays that hold 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=U64) & _M32 for c in (c0, c1, c2, c3))
    k0, k1 = key0 & 0xFFFFFFFF, key1 & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = c0 * U64(M0)          # < 2^64: exact
        p1 = c2 * U64(M1)
        hi0, lo0 = p0 >> U64(32), p0 & _M32
        hi1, lo1 = p1 >> U64(32), p1 & _M32
        c0, c1, c2, c3 = hi1 ^ c1 ^ U64(k0), lo1, hi0 ^ c3 ^ U64(k1), lo0
    return c0, c1, c2, c3


def block(seed: int, nonce: int, g, tag: int, b: int):
    """The four words of block b of stream `tag` for element indices g."""
    g = np.asarray(g, dtype=U64)
    c0 = g & _M32
    c1 = ((g >> U64(32)) & U64(0xFFFF)) | U64(tag << 16) | U64(b << 24)
    c2 = np.full_like(g, nonce & 0xFFFFFFFF)
    c3 = np.full_like(g, (nonce >> 32) & 0xFFFFFFFF)
    return philox4x32_10(c0, c1, c2, c3, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def _words(seed, nonce, g, tag, count):
    """The first `count` words of a stream, shape (len(g), count)."""
    out = []
    for b in range((count + 3) // 4):
        out.extend(block(seed, nonce, g, tag, b))
    return np.stack(out[:count], axis=1)


SHUFFLE_CHUNK_MAX = 1 << 32       # the largest product of radices one 64-bit chunk carries


def shuffle_radices(n: int):
    """Radices of the shuffle's n digits: t, then j_1 .. j_{n-1}."""
    return [2] + [i + 1 for i in range(1, n)]


def shuffle_chunks(n: int):
    """For each 64-bit chunk, the indices of the digits cut from it."""
    chunks, cur, prod = [], [], 1
    for k, m in enumerate(shuffle_radices(n)):
        if prod * m > SHUFFLE_CHUNK_MAX:
            chunks.append(cur)
            cur, prod = [], 1
        cur.append(k)
        prod *= m
    chunks.append(cur)
    return chunks


def chunk_digits(lo, hi, radices):
    """Digits of radices m_1, m_2, ... cut from the 64-bit fractions
    F = lo | hi << 32 (uint64 arrays of 32-bit words): F times m, the part
    above 2^64 is the digit and the rest the next F.  The 64 x 6-bit product
    is formed in two 32-bit halves, each exact in uint64."""
    lo = np.asarray(lo, dtype=U64).copy()
    hi = np.asarray(hi, dtype=U64).copy()
    out = []
    for m in radices:
        m = U64(m)
        p_lo = lo * m                              # < 2^38
        p_hi = hi * m + (p_lo >> U64(32))          # < 2^39
        lo, hi = p_lo & _M32, p_hi & _M32
        out.append(p_hi >> U64(32))
    return out


def shuffle_digits(seed01: int, nonce: int, g, n: int):
    """The n shuffle digits per element (shape (len(g), n))."""
    chunks = shuffle_chunks(n)
    radix = shuffle_radices(n)
    w = _words(seed01, nonce, g, TAG_SHUFFLE, 2 * len(chunks))
    digits = np.zeros((w.shape[0], n), dtype=U64)
    for c, idx in enumerate(chunks):
        for k, d in zip(idx, chunk_digits(w[:, 2 * c], w[:, 2 * c + 1], [radix[k] for k in idx])):
            digits[:, k] = d
    return digits


def fisher_yates(digits):
    """sigma (shape (len, n)) from the digits j_1 .. j_{n-1} (columns 1..):
    the inside-out shuffle A[i] = A[j_i], A[j_i] = i."""
    digits = np.asarray(digits)
    rows = np.arange(digits.shape[0])
    n = digits.shape[1]
    a = np.zeros((digits.shape[0], n), dtype=np.int64)
    for i in range(1, n):
        j = digits[:, i].astype(np.int64)
        a[:, i] = a[rows, j]
        a[rows, j] = i
    return a


def draw_shuffle(seed01: int, nonce: int, g, n: int):
    """t (uint64 0/1 per element) and sigma (shape (len(g), n)): sigma[:, s]
    is the window position placed in slot s by the shuffle of Alg. 7."""
    digits = shuffle_digits(seed01, nonce, g, n)
    return digits[:, 0].copy(), fisher_yates(digits)


def stream_masks(n: int, p: int) -> bool:
    """Whether the N = n slots' r and z are N-bit fields of the TAG_MASK bit
    stream: the default prime with N >= 17 (below, N-bit fields would cost
    more bias than the 32-bit multiply-shift)."""
    return n >= 17 and p == default_prime(n - 1)


def mask_blocks(n: int, p: int) -> int:
    """Philox blocks of one element's masks and reshares."""
    if stream_masks(n, p):
        return -(-2 * n * n // 128)
    return n if p >= (1 << 32) else (n + 1) // 2


def draw_masks(seed01: int, nonce: int, g, n: int, p: int):
    """r (in Z_p^*) and z (in Z_p), shape (N, n), indexed by slot."""
    g = np.asarray(g, dtype=U64)
    if stream_masks(n, p):
        w = _words(seed01, nonce, g, TAG_MASK, 4 * mask_blocks(n, p))
        w = np.concatenate([w, np.zeros((g.size, 1), dtype=U64)], axis=1)   # a zero word past the end
        r = np.empty((g.size, n), dtype=U64)
        z = np.empty((g.size, n), dtype=U64)
        for v in range(2 * n):
            off = n * v                                   # the field's first bit in the stream
            k, sh = off // 32, off % 32
            pair = w[:, k] | (w[:, k + 1] << U64(32))     # bits [32k, 32k + 64); the field ends below 32k + 64
            f = (pair >> U64(sh)) & U64((1 << n) - 1)
            if v % 2 == 0:
                r[:, v // 2] = np.minimum(np.maximum(f, U64(1)), U64(p - 1))
            else:
                z[:, v // 2] = f % U64(p)
        if p >= (1 << 32):                                # Python integers, as for the 64-bit words below
            return r.astype(object), z.astype(object)
        return r, z
    if p < (1 << 32):
        w = _words(seed01, nonce, g, TAG_MASK, 2 * n)
        R, Z = w[:, 0::2], w[:, 1::2]
        r = U64(1) + ((R * U64(p - 1)) >> U64(32))
        z = (Z * U64(p)) >> U64(32)
        return r, z
    r = np.empty((g.size, n), dtype=object)
    z = np.empty((g.size, n), dtype=object)
    for s in range(n):
        b = block(seed01, nonce, g, TAG_MASK, s)
        R = b[0].astype(object) | (b[1].astype(object) << 32)
        Z = b[2].astype(object) | (b[3].astype(object) << 32)
        r[:, s] = 1 + ((R * (p - 1)) >> 64)
        z[:, s] = (Z * p) >> 64
    return r, z


def _u64_pair(lo, hi):
    return lo | (hi << U64(32))


def draw_rho(seed02: int, nonce: int, g, ell: int):
    b = block(seed02, nonce, g, TAG_RESP, 0)
    return red(_u64_pair(b[0], b[1]), ell)


def draw_beaver(seed02: int, seed12: int, nonce: int, g, ell: int, tag: int = TAG_BEAVER):
    """([a]_0, [b]_0, [c]_0) from seed_02 and ([a]_1, [b]_1) from seed_12."""
    b0 = block(seed02, nonce, g, tag, 0)
    b1 = block(seed02, nonce, g, tag, 1)
    b2 = block(seed12, nonce, g, tag, 0)
    a0 = red(_u64_pair(b0[0], b0[1]), ell)
    bb0 = red(_u64_pair(b0[2], b0[3]), ell)
    c0 = red(_u64_pair(b1[0], b1[1]), ell)
    a1 = red(_u64_pair(b2[0], b2[1]), ell)
    bb1 = red(_u64_pair(b2[2], b2[3]), ell)
    return a0, bb0, c0, a1, bb1


def draw_rss(seed012: int, seed12: int, seed2: int, nonce: int, g, ell: int, relu: bool):
    """The replicated-sharing draws of Alg. drelu2's preprocessing (and of
    the ReLU's product): a dict with alpha (3 arrays), s1, s2, s (0/1),
    alpha_st (3) and, for the ReLU, alpha_relu (3)."""
    g = np.asarray(g, dtype=U64)
    nv = 10 if relu else 7
    w = _words(seed012, nonce, g, TAG_RSS, 2 * nv)
    v = [red(_u64_pair(w[:, 2 * k], w[:, 2 * k + 1]), ell) for k in range(nv)]
    b12 = block(seed12, nonce, g, TAG_RSS, 0)
    b2 = block(seed2, nonce, g, TAG_RSS, 0)
    out = {"alpha": v[0:3], "s1": v[3], "s2": red(_u64_pair(b12[0], b12[1]), ell), "s": b2[0] & U64(1),
           "alpha_st": v[4:7]}
    if relu:
        out["alpha_relu"] = v[7:10]
    return out
