"""Pins of the oracle's DReLU (Alg. 7) and ReLU (Alg. 8).

Independent of the oracle's code, the sign test is fixed by a closed form
derived from the sign-pattern theorem of Sec. 5.2 (Lemmas 3-5 in the
appendix) together with the exact e0 of deterministic truncation:

  x_t = (-1)^t x (signed),  R'_t = (-1)^t R' with [x]_0 = x + R', [x]_1 = -R',
  y_t = floor(x_t / 2^k_lo),
  c0  = [(x_t mod 2^k_lo) + (R'_t mod 2^k_lo) >= 2^k_lo]   (0 when k_lo = 0),
  D'  = 1 if y_t >= 1,  0 if y_t <= -1,  c0 if y_t = 0,
  DReLU = D' xor t,  ReLU = x * DReLU (x at full precision, Sec. 6.1),

exact for every R and t on the domain -ceil((2^(l_x+1) - 2)/3) < y_t <= 2^l_x
(upper end exclusive when k_lo > 0: a carry out of the dropped low bits can then
lift y_t = 2^l_x past the window; both ends were found by exhaustive search).
So outside the key-bit band |x| < 2^k_lo the reconstructed DReLU is the sign
bit [x > 0], and DReLU(0) = t when k_lo = 0 (the paper leaves it undefined).

Round-1 messages: after masking by r and resharing by z P2 must see
exactly as many zeros as there are zero adjacent sums v_i (zeros are kept,
non-zeros stay non-zero, Sec. 5.3); the count is predicted from the closed
form of each window u_i = floor(x_t / 2^(k_lo+i)) + e0_i.  The shuffle and
masks are checked statistically: the slot of the zero and the non-zero
masked values are uniform, each share is uniform on Z_p.
"""

import numpy as np
import pytest

from oracle import philox, protocols as P, ring
from oracle.params import default_prime

from closed_forms import expected_dprime, expected_zero_count, in_exact_domain

U = np.uint64


# ------------------------------------------------------------- helpers


def _random_randomness(rng, N, n, p, ell):
    sigma = np.argsort(rng.random((N, n)), axis=1)
    r = rng.integers(1, p, size=(N, n)).astype(U)
    z = rng.integers(0, p, size=(N, n)).astype(U)
    rho = rng.integers(0, 1 << 62, size=N).astype(U) * U(4) % U(1 << ell) if ell < 64 else \
        rng.integers(0, 1 << 63, size=N, dtype=np.uint64) * U(2)
    return sigma, r, z, ring.red(rho, ell)


def _zero_slots(w0, w1, p):
    w = (w0.astype(object) + w1.astype(object)) % p
    return w == 0


ELL8_CASES = [(lx, k) for lx in (3, 4) for k in range(0, 3) if k + 2 * lx <= 8]


@pytest.mark.parametrize("lx,k_lo", ELL8_CASES)
@pytest.mark.parametrize("t", [0, 1])
def test_drelu_exhaustive_l8(lx, k_lo, t):
    """Every x and every mask R at l = 8, both flips t, random shuffle/masks/rho."""
    ell = 8
    p = default_prime(lx)
    n = lx + 1
    x, R = np.meshgrid(np.arange(256, dtype=U), np.arange(256, dtype=U), indexing="ij")
    x, R = x.ravel(), R.ravel()
    x0, x1 = ring.split(x, R, ell)
    N = x.size
    tt = np.full(N, t, dtype=U)
    rng = np.random.default_rng(100 * lx + 10 * k_lo + t)
    sigma, r, z, rho = _random_randomness(rng, N, n, p, ell)
    y0, y1, w0, w1 = P.drelu_core(x0, x1, ell, lx, k_lo, p, tt, sigma, r, z, rho)
    y = ring.add(y0, y1, ell)
    dp = expected_dprime(x, R, tt, ell, k_lo)
    dom = in_exact_domain(x, tt, ell, lx, k_lo)
    assert dom.sum() > 0
    assert np.array_equal(y[dom], (dp ^ tt)[dom])
    # messages: zero count predicted by the per-window closed form, for every x
    zc = _zero_slots(w0, w1, p).sum(axis=1)
    assert np.array_equal(zc, expected_zero_count(x, R, tt, ell, lx, k_lo))
    # outputs canonical
    assert int(y0.max()) < 256 and int(y1.max()) < 256
    assert int(w0.max()) < p and int(w1.max()) < p


@pytest.mark.parametrize("lx,k_lo", ELL8_CASES)
def test_relu_exhaustive_l8(lx, k_lo):
    ell = 8
    p = default_prime(lx)
    n = lx + 1
    x, R = np.meshgrid(np.arange(256, dtype=U), np.arange(256, dtype=U), indexing="ij")
    x, R = x.ravel(), R.ravel()
    x0, x1 = ring.split(x, R, ell)
    N = x.size
    rng = np.random.default_rng(7 + lx + k_lo)
    tt = rng.integers(0, 2, size=N).astype(U)
    sigma, r, z, _ = _random_randomness(rng, N, n, p, ell)
    a0, b0, c0, a1, b1 = (rng.integers(0, 256, size=N).astype(U) for _ in range(5))
    y0, y1, _, _ = P.relu_core(x0, x1, ell, lx, k_lo, p, tt, sigma, r, z, a0, b0, c0, a1, b1)
    y = ring.add(y0, y1, ell)
    drelu = expected_dprime(x, R, tt, ell, k_lo) ^ tt
    dom = in_exact_domain(x, tt, ell, lx, k_lo)
    assert np.array_equal(y[dom], ring.mul(x, drelu, ell)[dom])
    # the Beaver identity holds for every x against the protocol's own bit
    d0, d1, _, _ = P.drelu_core(x0, x1, ell, lx, k_lo, p, tt, sigma, r, z, np.zeros(N, U))
    assert np.array_equal(y, ring.mul(x, ring.add(d0, d1, ell), ell))


SAMPLED = [  # (ell, lx, k_lo): rings 12 and 16, and the l = 64 settings of the workloads
    (12, 4, 2), (12, 5, 1), (16, 6, 4), (16, 5, 5),
    (64, 7, 11), (64, 18, 13), (64, 31, 0), (64, 32, 0), (51, 11, 13), (24, 7, 10), (32, 8, 8),
]


@pytest.mark.parametrize("ell,lx,k_lo", SAMPLED)
def test_drelu_relu_sampled_with_prg(ell, lx, k_lo):
    """Full Alg. 7 / Alg. 8 with the seeded draws, random x inside the guard domain."""
    p = default_prime(lx)
    rng = np.random.default_rng(ell * 1000 + lx * 10 + k_lo)
    N = 3000
    bound = 1 << (k_lo + lx - 1)
    xs = rng.integers(-bound + 1, bound, size=N)
    xs[:50] = rng.integers(-(1 << k_lo), (1 << k_lo) + 1, size=50)      # the key-bit band
    xs[50] = 0
    x = np.array([v % (1 << ell) for v in xs.tolist()], dtype=U)
    R = ring.red(rng.integers(0, 1 << 63, size=N, dtype=np.uint64) * U(2) + U(1), ell)
    x0, x1 = ring.split(x, R, ell)
    seeds = (0x1234_5678_9ABC_DEF0 + ell, 0x0FED_CBA9_8765_4321, 0x1111_2222_3333_4444 + lx)
    nonce = 0xABCDEF + k_lo
    y0, y1, w0, w1 = P.drelu(x0, x1, ell, lx, k_lo, p, seeds, nonce)
    g = np.arange(N, dtype=U)
    t, _ = philox.draw_shuffle(seeds[0], nonce, g, lx + 1)
    dp = expected_dprime(x, R, t, ell, k_lo)
    y = ring.add(y0, y1, ell)
    assert np.array_equal(y, dp ^ t)
    outside = np.abs(xs) >= (1 << k_lo)
    assert np.array_equal(y[outside], (xs[outside] > 0).astype(U))
    if k_lo == 0:
        assert int(y[50]) == int(t[50])
    zc = _zero_slots(w0, w1, p).sum(axis=1)
    assert np.array_equal(zc[:400], expected_zero_count(x[:400], R[:400], t[:400], ell, lx, k_lo))
    r0, r1, _, _ = P.relu(x0, x1, ell, lx, k_lo, p, seeds, nonce)
    assert np.array_equal(ring.add(r0, r1, ell), ring.mul(x, dp ^ t, ell))


def test_drelu_randomness_is_element_local():
    """Same element, same seeds/nonce -> same outputs and messages whether it is
    evaluated alone or inside a larger batch (counter = global element index)."""
    ell, lx, k_lo = 64, 7, 11
    p = default_prime(lx)
    rng = np.random.default_rng(1)
    N = 500
    x = ring.red(rng.integers(-(1 << 16), 1 << 16, size=N).astype(np.int64).astype(U), ell)
    R = rng.integers(0, 1 << 63, size=N, dtype=np.uint64)
    x0, x1 = ring.split(x, R, ell)
    seeds = (5, 6, 7)
    full = P.relu(x0, x1, ell, lx, k_lo, p, seeds, 9, elem_base=1000)
    part = P.relu(x0[200:300], x1[200:300], ell, lx, k_lo, p, seeds, 9, elem_base=1200)
    for a, b in zip(full, part):
        assert np.array_equal(a[200:300], b)


# ------------------------------------------- hiding: shuffle, masks, reshare


def _chi2_ok(counts, dof_sigma=6.0):
    counts = np.asarray(counts, dtype=float)
    e = counts.sum() / counts.size
    chi2 = ((counts - e) ** 2 / e).sum()
    dof = counts.size - 1
    return abs(chi2 - dof) <= dof_sigma * np.sqrt(2 * dof)


def test_zero_slot_uniform_and_masked_values_uniform():
    """For a fixed positive x, P2 sees exactly one zero among n slots; its slot is uniform
    (the shuffle hides the bit position) and the other reconstructed w_j are uniform
    on Z_p^* (the mask r); each single share w0_j is uniform on Z_p (the reshare z)."""
    ell, lx, k_lo = 64, 7, 0
    p = default_prime(lx)
    n = lx + 1
    N = 40000
    x = np.full(N, 37, dtype=U)
    rng = np.random.default_rng(2)
    R = rng.integers(0, 1 << 63, size=N, dtype=np.uint64)
    x0, x1 = ring.split(x, R, ell)
    _, _, w0, w1 = P.drelu(x0, x1, ell, lx, k_lo, p, (11, 12, 13), 77)
    zs = _zero_slots(w0, w1, p)
    g = np.arange(N, dtype=U)
    t, _ = philox.draw_shuffle(11, 77, g, n)
    pos = t == 0                                        # unflipped: x > 0 -> zeros present
    assert np.all(zs[pos].sum(axis=1) >= 1) and np.all(zs[~pos].sum(axis=1) == 0)
    single = pos & (zs.sum(axis=1) == 1)
    slot = np.argmax(zs[single], axis=1)
    assert _chi2_ok(np.bincount(slot, minlength=n))
    w = ((w0.astype(object) + w1.astype(object)) % p).astype(np.int64)
    nonzero = w[~zs]
    assert nonzero.min() >= 1
    assert _chi2_ok(np.bincount(nonzero, minlength=p)[1:])
    assert _chi2_ok(np.bincount(w0.astype(np.int64).ravel(), minlength=p))


def test_msg_bits_tab1(golden):
    for ell, lx, bits, rounds, *_ in golden("tab1_comm.txt"):
        ell, lx = int(ell), int(lx)
        b, r = P.msg_bits("drelu", ell, lx, default_prime(lx))
        assert b[0] == b[1] == int(bits) and r == int(rounds)
    b, r = P.msg_bits("relu", 64, 7, 251)
    assert b == [64, 64, 64, 128, 64, 64] and r == 2
