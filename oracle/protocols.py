"""The paper's share-local protocols, written out plainly (test infrastructure only).

Shares are NumPy uint64 arrays with canonical values.  Party P_j holds
[x]_j; all three parties are evaluated here side by side, and each step is
labelled with the party that performs it.

Readings of the paper taken here, where it is silent or ambiguous:
* Alg. 1 / Alg. 4 / Alg. 5, P1's share: 2^l - [x]_1 is reduced mod 2^l
  before the cut, i.e. P1 cuts -[x]_1 mod 2^l (the worked examples of Sec. 1
  and Sec. 5.1 write cut(-[x]_1, .)).
* Alg. 5 input: k1 low bits and k2 high bits are dropped (the worked example
  of Sec. 5.1 with k1 = 4, k2 = 1 fixes this; the algorithm's statement of
  its input has the two words swapped).
* Alg. 7 windows with key bits (Sec. 6.1): window i is trc(x, k_lo+i,
  l-l_x-k_lo-i), i = 0..l_x.
* Alg. 7 adjacent sums: the constant -1 is added by P0 only; u_{l_x+1} := 0.
* Alg. 7 shuffle, mask and reshare: r_i and z_i are indexed by the slot
  after the shuffle; the reshare is w0 += z, w1 -= z with z uniform in Z_p
  from seed_01.
* Alg. 7 reply: P2 shares its bit as (rho, D' - rho) with rho from seed_02.
* Alg. 7 unflip and Alg. 8's product: P0 adds the public constants (t, de).
* Alg. 8: [c]_1 is sent once, in preprocessing; the d-shares are exchanged
  between P0 and P1.
* Alg. linear (truncate-then-multiply): the truncation is Alg. 1; with an
  odd f the first factor drops floor(f/2) bits and the second ceil(f/2).
  The product is a Beaver multiplication with the triple dealt as in
  Alg. 8's preprocessing ([a]_0, [b]_0, [c]_0 from seed_02, [a]_1, [b]_1
  from seed_12, [c]_1 formed by P2), under its own stream tag.
* Alg. drelu2 (replicated sharing, appendix): x = [x]_0 + [x]_1 + [x]_2 and
  P_j holds ([x]_j, [x]_{j+1}), indices mod 3 (the shares each party forms in
  the preprocessing say so).  Every party draws all three alpha_j from
  seed_012.  The products [s][t] and, for the ReLU, [x][DReLU(x)] use the
  replicated-sharing multiplication: P_j forms
  z_j = u_j v_j + u_j v_{j+1} + u_{j+1} v_j + gamma_j with a zero sharing
  gamma_j = alpha'_j - alpha'_{j-1} (fresh alphas from seed_012, built like
  the sharing of t) and sends z_j to P_{j-1}; the product's shares are z_j.
  The public bit D'' is added to share 0 (held by P0 and P2), and is counted
  as an l-bit value, as the algorithm reduces it mod 2^l.
"""

import numpy as np

from . import philox
from .params import check_drelu
from .ring import U64, add, cut, mul, neg, red, sub


# ---------------------------------------------------------------- truncation


def trunc_prob(x0, x1, ell: int, k: int):
    """Alg. 1 (SecureML truncation): outputs in Z_{2^l}.

    P0: cut([x]_0, k) mod 2^l.   P1: 2^l - cut(2^l - [x]_1, k) mod 2^l.
    """
    y0 = red(cut(x0, k, 0, ell), ell)
    y1 = neg(cut(neg(x1, ell), k, 0, ell), ell)
    return y0, y1


def trunc_det(x0, x1, ell: int, k1: int, k2: int = 0):
    """Alg. 4 (k2 = 0) and Alg. 5: outputs in Z_{2^(l-k1-k2)}.

    P0: cut([x]_0, k1, k2) mod 2^(l-k1-k2).
    P1: 2^l - cut(2^l - [x]_1, k1, k2) mod 2^(l-k1-k2).
    """
    m = ell - k1 - k2
    if not (0 <= k1 and 0 <= k2 and m >= 1):
        raise ValueError("need k1, k2 >= 0 and k1 + k2 < l")
    y0 = cut(x0, k1, k2, ell)
    y1 = neg(cut(neg(x1, ell), k1, k2, ell), m)
    return y0, y1


# -------------------------------------------------------------- modulo switch


def mod_switch(a0, a1, ell_in: int, p: int):
    """Alg. 6: shares in Z_{2^l'} -> shares in Z_p, log2 p = l' + 1.

    P0: 2^l' mod p if [x]_0 = 0, else [x]_0 mod p.
    P1: p + [x]_1 - 2^l' mod p.
    Works elementwise on arrays of any shape.
    """
    a0 = red(a0, ell_in).astype(object)
    a1 = red(a1, ell_in).astype(object)
    two = pow(2, ell_in, p)
    s0 = np.where(a0 == 0, two, a0 % p)
    s1 = (p + a1 - (1 << ell_in)) % p
    if p < (1 << 63):
        return s0.astype(U64), s1.astype(U64)
    return s0, s1


def _mulmod(a, b, p):
    if p < (1 << 32):
        return (np.asarray(a, dtype=U64) * np.asarray(b, dtype=U64)) % U64(p)
    return (np.asarray(a, dtype=object) * np.asarray(b, dtype=object)) % p


# -------------------------------------------------------------------- DReLU


def drelu_round1(x0, x1, ell, lx, k_lo, p, t, sigma, r, z):
    """Alg. 7 for P0 and P1 up to their first message: the messages [w]_0, [w]_1 (N x n,
    in slot order) that they send to P2."""
    check_drelu(ell, lx, k_lo, p)
    n = lx + 1
    x0, x1 = red(x0, ell), red(x1, ell)
    N = x0.size
    flip = np.asarray(t, dtype=U64).astype(bool)
    # flip (P0, P1): [x] := (-1)^t [x]
    a0 = np.where(flip, neg(x0, ell), x0)
    a1 = np.where(flip, neg(x1, ell), x1)
    # windows (P0, P1): u_i = trc(x, k_lo+i, l-l_x-k_lo-i), i = 0..l_x
    u0 = np.zeros((N, n + 1), dtype=U64)      # column n is u_{l_x+1} := 0
    u1 = np.zeros((N, n + 1), dtype=U64)
    for i in range(n):
        k1 = k_lo + i
        u0[:, i], u1[:, i] = trunc_det(a0, a1, ell, k1, ell - lx - k1)
    # adjacent sums: v_i = u_i + u_{i+1} - 1 (P0 subtracts the 1), mod 2^l_x
    v0 = red(u0[:, :n] + u0[:, 1:] - U64(1), lx)
    v1 = red(u1[:, :n] + u1[:, 1:], lx)
    # modulo switch: Alg. 6 on every v_i
    s0, s1 = mod_switch(v0, v1, lx, p)
    # shuffle with seed_01; slot j receives position sigma[:, j]
    s0 = np.take_along_axis(s0, sigma, axis=1)
    s1 = np.take_along_axis(s1, sigma, axis=1)
    # mask with r_j in Z_p^* (same r for both parties)
    w0 = _mulmod(s0, r, p)
    w1 = _mulmod(s1, r, p)
    # reshare with z_j and send to P2
    if p < (1 << 32):
        z = np.asarray(z, dtype=U64)
        w0 = (w0 + z) % U64(p)
        w1 = (w1 + (U64(p) - z)) % U64(p)
    else:
        w0 = (w0 + z) % p
        w1 = (w1 - z) % p
    return w0, w1


def p2_zero_test(w0, w1, p):
    """Alg. 7, P2's zero test: reconstruct w_j and set D' = 1 iff some w_j = 0."""
    if p < (1 << 32):
        w = (np.asarray(w0, dtype=U64) + np.asarray(w1, dtype=U64)) % U64(p)
    else:
        w = (np.asarray(w0, dtype=object) + np.asarray(w1, dtype=object)) % p
    return np.any(w == 0, axis=1).astype(U64)


def drelu_core(x0, x1, ell, lx, k_lo, p, t, sigma, r, z, rho):
    """Alg. 7 with the random values passed in.  Returns (y0, y1, w0, w1)."""
    w0, w1 = drelu_round1(x0, x1, ell, lx, k_lo, p, t, sigma, r, z)
    dp = p2_zero_test(w0, w1, p)
    # reply (P2): respond with a fresh sharing of D' in Z_{2^l}
    d0 = red(rho, ell)
    d1 = sub(dp, d0, ell)
    # unflip (P0, P1): DReLU = D' xor t = t + (1-2t) D'
    flip = np.asarray(t, dtype=U64).astype(bool)
    y0 = np.where(flip, sub(U64(1), d0, ell), d0)
    y1 = np.where(flip, neg(d1, ell), d1)
    return y0, y1, w0, w1


def relu_core(x0, x1, ell, lx, k_lo, p, t, sigma, r, z, a0, b0, c0, a1, b1):
    """Alg. 8 (UBL ReLU) with the random values passed in.

    Returns (y0, y1, w0, w1)."""
    x0, x1 = red(x0, ell), red(x1, ell)
    # preprocessing (P2): [c]_1 = ([a]_0 + [a]_1)([b]_0 + [b]_1) - [c]_0
    c1 = sub(mul(add(a0, a1, ell), add(b0, b1, ell), ell), c0, ell)
    # Alg. 7 up to the parties' first message, then P2's zero test
    w0, w1 = drelu_round1(x0, x1, ell, lx, k_lo, p, t, sigma, r, z)
    dp = p2_zero_test(w0, w1, p)
    # P2: e = D' - b
    e = sub(dp, add(b0, b1, ell), ell)
    # P0, P1: d = x - a, reconstructed from both parties' shares
    d = add(sub(x0, a0, ell), sub(x1, a1, ell), ell)
    # product: [x D'] = de + d[b] + e[a] + [c];  ReLU = t[x] + (1-2t)[x D']
    m0 = add(add(add(mul(d, e, ell), mul(d, b0, ell), ell), mul(e, a0, ell), ell), c0, ell)
    m1 = add(add(mul(d, b1, ell), mul(e, a1, ell), ell), c1, ell)
    flip = np.asarray(t, dtype=U64).astype(bool)
    y0 = np.where(flip, sub(x0, m0, ell), m0)
    y1 = np.where(flip, sub(x1, m1, ell), m1)
    return y0, y1, w0, w1


def _indices(n_elems, elem_base, g):
    if g is not None:
        return np.asarray(g, dtype=U64)
    return U64(elem_base) + np.arange(n_elems, dtype=U64)


def drelu(x0, x1, ell, lx, k_lo, p, seeds, nonce, elem_base=0, g=None):
    """Alg. 7 with randomness drawn from the seeds (see ``philox``).

    seeds = (seed_01, seed_02, seed_12); g = global element indices (default
    elem_base + arange(N)).  Returns (y0, y1, w0, w1)."""
    seed01, seed02, _ = seeds
    g = _indices(np.asarray(x0).size, elem_base, g)
    n = lx + 1
    t, sigma = philox.draw_shuffle(seed01, nonce, g, n)
    r, z = philox.draw_masks(seed01, nonce, g, n, p)
    rho = philox.draw_rho(seed02, nonce, g, ell)
    return drelu_core(x0, x1, ell, lx, k_lo, p, t, sigma, r, z, rho)


def relu(x0, x1, ell, lx, k_lo, p, seeds, nonce, elem_base=0, g=None):
    """Alg. 8 with randomness drawn from the seeds.  Returns (y0, y1, w0, w1)."""
    seed01, seed02, seed12 = seeds
    g = _indices(np.asarray(x0).size, elem_base, g)
    n = lx + 1
    t, sigma = philox.draw_shuffle(seed01, nonce, g, n)
    r, z = philox.draw_masks(seed01, nonce, g, n, p)
    a0, b0, c0, a1, b1 = philox.draw_beaver(seed02, seed12, nonce, g, ell)
    return relu_core(x0, x1, ell, lx, k_lo, p, t, sigma, r, z, a0, b0, c0, a1, b1)


# ------------------------------- parties apart: packed round-1 messages (Alg. 7)


def msg_words(npos: int) -> int:
    """32-bit words per element of one party's packed round-1 message: npos
    slots of npos bits each (p has npos = l_x + 1 bits), rounded up."""
    return (npos * npos + 31) // 32


def pack_messages(w, npos: int):
    """Bit-pack one party's messages (N x npos values < 2^npos, slot order):
    bit b of slot s is bit s * npos + b of the element's bit string, and word
    k holds its bits 32k .. 32k + 31.  Returns uint32 words, word-major:
    out[k, i] is word k of element i."""
    w = np.asarray(w, dtype=object)
    N = w.shape[0]
    out = np.zeros((msg_words(npos), N), dtype=object)
    for s in range(npos):
        for b in range(npos):
            pos = s * npos + b
            out[pos // 32] += ((w[:, s] >> b) & 1) << (pos % 32)
    return out.astype(np.uint32)


def unpack_messages(words, npos: int):
    """Inverse of ``pack_messages``: N x npos slot values (Python ints)."""
    words = np.asarray(words, dtype=np.uint32).astype(object)
    N = words.shape[1]
    w = np.zeros((N, npos), dtype=object)
    for s in range(npos):
        for b in range(npos):
            pos = s * npos + b
            w[:, s] += ((words[pos // 32] >> (pos % 32)) & 1) << b
    return w


def drelu_send(party, xj, ell, lx, k_lo, p, seeds, nonce, elem_base=0, g=None):
    """P0's or P1's part of Alg. 7's first round with its own share only: the
    packed message it sends to P2.  Every step before P2 is share-local, so
    the other party's share does not enter; it is passed to drelu_round1 as
    zero and that party's output is dropped."""
    xj = np.asarray(xj, dtype=U64)
    g = _indices(xj.size, elem_base, g)
    n = lx + 1
    t, sigma = philox.draw_shuffle(seeds[0], nonce, g, n)
    r, z = philox.draw_masks(seeds[0], nonce, g, n, p)
    zero = np.zeros_like(xj)
    w0, w1 = drelu_round1(xj if party == 0 else zero, xj if party == 1 else zero, ell, lx, k_lo, p, t, sigma, r, z)
    return pack_messages(w0 if party == 0 else w1, n)


def drelu_reply(words0, words1, ell, lx, p, seeds, nonce, elem_base=0, g=None):
    """P2: unpack both messages, D' = [some slot reconstructs to 0], and the
    reply shares (rho, D' - rho) of Z_{2^l} for P0 and P1."""
    w0, w1 = unpack_messages(words0, lx + 1), unpack_messages(words1, lx + 1)
    g = _indices(w0.shape[0], elem_base, g)
    dp = p2_zero_test(w0, w1, p)
    rho = philox.draw_rho(seeds[1], nonce, g, ell)
    return rho, sub(dp, rho, ell)


def drelu_finish(party, dj, ell, lx, seeds, nonce, elem_base=0, g=None):
    """P0 or P1 unflips its reply share: P0 t + (1 - 2t) d0, P1 (1 - 2t) d1."""
    dj = np.asarray(dj, dtype=U64)
    g = _indices(dj.size, elem_base, g)
    t, _ = philox.draw_shuffle(seeds[0], nonce, g, lx + 1)
    flip = t.astype(bool)
    if party == 0:
        return np.where(flip, sub(U64(1), dj, ell), red(dj, ell))
    return np.where(flip, neg(dj, ell), red(dj, ell))


# -------------------------------------- truncate-then-multiply (Alg. linear)

TRUNC_NONE, TRUNC_AFTER, TRUNC_BEFORE = 0, 1, 2


def beaver_mul(x0, x1, y0, y1, ell, a0, b0, c0, a1, b1):
    """[x y] from 2-of-2 shares and a Beaver triple.  P2 forms
    [c]_1 = (a0 + a1)(b0 + b1) - c0 and sends it to P1; P0 and P1 open
    d = x - a and e = y - b; [xy]_0 = de + d[b]_0 + e[a]_0 + [c]_0 and
    [xy]_1 = d[b]_1 + e[a]_1 + [c]_1."""
    c1 = sub(mul(add(a0, a1, ell), add(b0, b1, ell), ell), c0, ell)
    d = add(sub(x0, a0, ell), sub(x1, a1, ell), ell)
    e = add(sub(y0, b0, ell), sub(y1, b1, ell), ell)
    z0 = add(add(add(mul(d, e, ell), mul(d, b0, ell), ell), mul(e, a0, ell), ell), c0, ell)
    z1 = add(add(mul(d, b1, ell), mul(e, a1, ell), ell), c1, ell)
    return z0, z1


def mul_trunc_core(x0, x1, y0, y1, ell, f, order, a0, b0, c0, a1, b1):
    """The product of two shared values with f fractional bits dropped:
    order TRUNC_BEFORE is Alg. linear (Alg. 1 on x by floor(f/2) bits and on
    y by ceil(f/2), then the product); TRUNC_AFTER multiplies, then applies
    Alg. 1 by f; TRUNC_NONE (f = 0) is the plain product."""
    x0, x1, y0, y1 = (red(v, ell) for v in (x0, x1, y0, y1))
    if order == TRUNC_BEFORE:
        x0, x1 = trunc_prob(x0, x1, ell, f // 2)
        y0, y1 = trunc_prob(y0, y1, ell, f - f // 2)
    z0, z1 = beaver_mul(x0, x1, y0, y1, ell, a0, b0, c0, a1, b1)
    if order == TRUNC_AFTER:
        z0, z1 = trunc_prob(z0, z1, ell, f)
    return z0, z1


def mul_trunc(x0, x1, y0, y1, ell, f, order, seeds, nonce, elem_base=0, g=None):
    """``mul_trunc_core`` with the triple drawn from the seeds (seed_02,
    seed_12 of seeds = (seed_01, seed_02, seed_12, ...))."""
    g = _indices(np.asarray(x0).size, elem_base, g)
    a0, b0, c0, a1, b1 = philox.draw_beaver(seeds[1], seeds[2], nonce, g, ell, tag=philox.TAG_MUL)
    return mul_trunc_core(x0, x1, y0, y1, ell, f, order, a0, b0, c0, a1, b1)


# ----------------------------------- replicated secret sharing (Alg. drelu2)


def rss_reconstruct(sh, ell):
    """x = [x]_0 + [x]_1 + [x]_2 mod 2^l."""
    return add(add(sh[0], sh[1], ell), sh[2], ell)


def zero_sharing(alpha, ell):
    """beta_j = alpha_j - alpha_{j-1} (indices mod 3): three shares of 0, as
    the preprocessing of Alg. drelu2 builds them from seed_012."""
    return [sub(alpha[j], alpha[j - 1], ell) for j in range(3)]


def rss_mul(u, v, gamma, ell):
    """[u v] from replicated shares: P_j holds (u_j, u_{j+1}), (v_j, v_{j+1})
    and forms z_j = u_j v_j + u_j v_{j+1} + u_{j+1} v_j + gamma_j; the nine
    cross terms u_a v_b each appear once over j = 0, 1, 2, and the gamma_j
    sum to 0.  P_j sends z_j to P_{j-1}, so that P_j holds (z_j, z_{j+1})."""
    z = []
    for j in range(3):
        k = (j + 1) % 3
        zj = add(add(mul(u[j], v[j], ell), mul(u[j], v[k], ell), ell), mul(u[k], v[j], ell), ell)
        z.append(add(zj, gamma[j], ell))
    return z


def rss_preprocess(t, d, ell):
    """Alg. drelu2 preprocessing, from t (seed_01) and the draws d of
    ``philox.draw_rss``.  Returns ([t], [s], [s xor t]), each a list of
    three share arrays."""
    t = np.asarray(t, dtype=U64)
    # [t] := (beta_0, beta_1 + t, beta_2) with beta_j = alpha_j - alpha_{j-1}
    beta = zero_sharing(d["alpha"], ell)
    ts = [beta[0], add(beta[1], t, ell), beta[2]]
    # [s]_1 from seed_012, [s]_2 from seed_12; P2 draws the bit s from seed_2
    # and sends [s]_0 = s - [s]_1 - [s]_2 to P0
    s0 = sub(sub(red(d["s"], ell), d["s1"], ell), d["s2"], ell)
    ss = [s0, d["s1"], d["s2"]]
    # [s xor t] = [s] + [t] - 2 [s][t]
    st = rss_mul(ss, ts, zero_sharing(d["alpha_st"], ell), ell)
    sxt = [sub(add(ss[j], ts[j], ell), mul(U64(2), st[j], ell), ell) for j in range(3)]
    return ts, ss, sxt


def rss_drelu_core(x, ell, lx, k_lo, p, t, sigma, r, z, d):
    """Alg. drelu2 with the random values passed in (t, sigma, r, z as for
    Alg. 7; d from ``philox.draw_rss``).  x = three share arrays.  Returns
    (y, w0, w1): y the three shares of DReLU(x), w0, w1 the round-1
    messages."""
    x = [red(xi, ell) for xi in x]
    _, _, sxt = rss_preprocess(t, d, ell)
    # P0 enters [x]_0 + [x]_1, P1 enters [x]_2; both run Alg. 7 up to their
    # messages to P2
    w0, w1 = drelu_round1(add(x[0], x[1], ell), x[2], ell, lx, k_lo, p, t, sigma, r, z)
    dp = p2_zero_test(w0, w1, p)
    # P2: D'' = s xor D', sent to P0 and P1
    dpp = dp ^ np.asarray(d["s"], dtype=U64)
    # everyone: [DReLU(x)] = D'' + [s xor t] - 2 D'' [s xor t]; the public
    # D'' goes to share 0
    y = [sub(sxt[j], mul(U64(2) * dpp, sxt[j], ell), ell) for j in range(3)]
    y[0] = add(y[0], dpp, ell)
    return y, w0, w1


def rss_relu_core(x, ell, lx, k_lo, p, t, sigma, r, z, d):
    """RSS ReLU (appendix): Alg. drelu2, then the replicated-sharing product
    [x][DReLU(x)] with the full-precision x.  Returns (y, w0, w1)."""
    x = [red(xi, ell) for xi in x]
    dr, w0, w1 = rss_drelu_core(x, ell, lx, k_lo, p, t, sigma, r, z, d)
    y = rss_mul(x, dr, zero_sharing(d["alpha_relu"], ell), ell)
    return y, w0, w1


def _rss(x0, x1, x2, ell, lx, k_lo, p, seeds, nonce, elem_base, g, relu):
    seed01, _, seed12, seed012, seed2 = seeds
    g = _indices(np.asarray(x0).size, elem_base, g)
    n = lx + 1
    t, sigma = philox.draw_shuffle(seed01, nonce, g, n)
    r, z = philox.draw_masks(seed01, nonce, g, n, p)
    d = philox.draw_rss(seed012, seed12, seed2, nonce, g, ell, relu)
    core = rss_relu_core if relu else rss_drelu_core
    return core((x0, x1, x2), ell, lx, k_lo, p, t, sigma, r, z, d)


def rss_drelu(x0, x1, x2, ell, lx, k_lo, p, seeds, nonce, elem_base=0, g=None):
    """Alg. drelu2 with randomness drawn from the seeds.

    seeds = (seed_01, seed_02, seed_12, seed_012, seed_2) (seed_02 is not
    drawn from).  Returns (y, w0, w1) with y = [y_0, y_1, y_2]."""
    return _rss(x0, x1, x2, ell, lx, k_lo, p, seeds, nonce, elem_base, g, False)


def rss_relu(x0, x1, x2, ell, lx, k_lo, p, seeds, nonce, elem_base=0, g=None):
    """RSS ReLU with randomness drawn from the seeds.  Returns (y, w0, w1)."""
    return _rss(x0, x1, x2, ell, lx, k_lo, p, seeds, nonce, elem_base, g, True)


# ------------------------------------------------------ message accounting

LINKS = ("P0->P2", "P1->P2", "P2->P0", "P2->P1", "P0->P1", "P1->P0")


def msg_bits(op: str, ell: int, lx: int, p: int):
    """Theoretical bits per element on each link, and the online rounds.

    Round 1: each of P0, P1 sends n = l_x + 1 values of Z_p, i.e.
    (l_x + 1) * ceil(log2 p) = (l_x + 1)^2 bits (Tab. 1, Sec. 5.4).
    DReLU round 2: one Z_{2^l} share to each of P0, P1.
    ReLU: e to P0 and P1, [c]_1 to P1 (preprocessing), d-shares both ways
    between P0 and P1 (concurrent with round 1, so still 2 rounds).
    """
    wbits = (lx + 1) * p.bit_length()
    if op == "drelu":
        return [wbits, wbits, ell, ell, 0, 0], 2
    if op == "relu":
        return [wbits, wbits, ell, 2 * ell, ell, ell], 2
    # Alg. drelu2: preprocessing sends [s]_0 (P2->P0) and the reshared z_j of
    # [s][t] (P0->P2, P1->P0, P2->P1); online, round 1 as Alg. 7 and D'' from
    # P2 to P0 and P1.  The RSS ReLU adds one more product: a third round.
    if op == "rss_drelu":
        return [wbits + ell, wbits, 2 * ell, 2 * ell, 0, ell], 2
    if op == "rss_relu":
        return [wbits + 2 * ell, wbits, 2 * ell, 3 * ell, 0, 2 * ell], 3
    raise ValueError(op)
