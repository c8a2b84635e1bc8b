"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

All arithmetic is integer, so the bar is equality of every output share and
every captured round-1 message (tolerance 0).  Sizes span several thread
blocks and a ragged tail; unaligned views exercise the scalar path of the
streaming kernels; element indices cross 2^32.
"""

import numpy as np
import pytest

from oracle import philox as OPH
from oracle import protocols as OPR
from oracle.params import default_prime
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop
    return bicop


def dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda()
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda()
    raise TypeError(a.dtype)


def host(t):
    t = t.detach().cpu()
    if t.element_size() == 8:
        return t.view(torch.int64).numpy().view(np.uint64)
    return t.view(torch.int32).numpy().view(np.uint32)


def same(a, b):
    """Bitwise equality of two integer tensors of the same element size."""
    def v(t):
        return t.view(torch.int64) if t.element_size() == 8 else t.view(torch.int32)
    return a.shape == b.shape and a.element_size() == b.element_size() and torch.equal(v(a), v(b))


def rand_ring(rng, n, ell):
    v = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    if ell < 64:
        v &= np.uint64((1 << ell) - 1)
    return v.astype(W.storage_dtype(ell))


SIZES = [1, 7, 256, 1023, 4097, 65537]


# --------------------------------------------------------------------- PRG


def test_prg_million_counters(B):
    """Raw Philox4x32-10 stream against the oracle's generator on 2^18
    elements x 4 blocks = 1,048,576 counters (4 Mi words), with element
    indices crossing 2^32 and a nonce and key with every word nonzero."""
    n, nb, tag = 1 << 18, 4, 2
    seed, nonce, base = 0xA5A5F00DC0FFEE11, 0x1122334455667788, (1 << 32) - (1 << 17)
    got = host(B.prg_blocks(n, nb, seed, nonce, tag, base)).reshape(n, nb, 4)
    g = np.arange(n, dtype=np.uint64) + np.uint64(base)
    for b in range(nb):
        exp = np.stack(OPH.block(seed, nonce, g, tag, b), axis=1).astype(np.uint32)
        assert np.array_equal(got[:, b, :], exp), b


@pytest.mark.parametrize("tag", [1, 2, 3, 4, 200])
def test_prg_blocks_match_oracle(B, tag):
    for elem_base, n, nb in [(0, 5000, 3), ((1 << 32) - 100, 300, 2), ((1 << 47) + 12345, 64, 9)]:
        seed, nonce = 0xDEADBEEF12345678 ^ tag, 0x0123456789ABCDEF + elem_base
        got = host(B.prg_blocks(n, nb, seed, nonce, tag, elem_base)).reshape(n, nb, 4)
        g = np.arange(n, dtype=np.uint64) + np.uint64(elem_base)
        for b in range(nb):
            exp = np.stack(OPH.block(seed, nonce, g, tag, b), axis=1).astype(np.uint32)
            assert np.array_equal(got[:, b, :], exp), (elem_base, b)


# ----------------------------------------------------------- streaming kernels


TRUNC_CASES = [(64, 13, 0), (64, 13, 5), (64, 40, 0), (64, 33, 8), (51, 13, 0), (40, 8, 0), (32, 8, 0),
               (32, 4, 4), (24, 3, 1), (16, 4, 0), (8, 4, 1), (63, 1, 61), (64, 0, 0)]


@pytest.mark.parametrize("ell,k1,k2", TRUNC_CASES)
def test_trunc_det_parity(B, ell, k1, k2):
    rng = np.random.default_rng(ell * 100 + k1 * 10 + k2)
    for n in SIZES:
        x0, x1 = rand_ring(rng, n, ell), rand_ring(rng, n, ell)
        y0, y1 = B.trunc_det(dev(x0), dev(x1), ell, k1, k2)
        e0, e1 = OPR.trunc_det(x0.astype(np.uint64), x1.astype(np.uint64), ell, k1, k2)
        assert np.array_equal(host(y0).astype(np.uint64), e0) and np.array_equal(host(y1).astype(np.uint64), e1)


@pytest.mark.parametrize("ell,k", [(64, 13), (64, 26), (64, 63), (51, 13), (32, 8), (20, 7), (8, 4)])
def test_trunc_prob_parity(B, ell, k):
    rng = np.random.default_rng(ell + k)
    for n in SIZES:
        x0, x1 = rand_ring(rng, n, ell), rand_ring(rng, n, ell)
        y0, y1 = B.trunc_prob(dev(x0), dev(x1), ell, k)
        e0, e1 = OPR.trunc_prob(x0.astype(np.uint64), x1.astype(np.uint64), ell, k)
        assert np.array_equal(host(y0).astype(np.uint64), e0) and np.array_equal(host(y1).astype(np.uint64), e1)


@pytest.mark.parametrize("ell", [2, 7, 11, 18, 24, 31, 32, 33, 40, 62])
def test_mod_switch_parity(B, ell):
    rng = np.random.default_rng(ell)
    p = default_prime(ell) if ell <= 32 else _prime_above(ell)
    for n in SIZES:
        x0, x1 = rand_ring(rng, n, ell), rand_ring(rng, n, ell)
        x0[: n // 4] = 0                                          # exercise the P0 zero case
        y0, y1 = B.mod_switch(dev(x0), dev(x1), ell, p)
        e0, e1 = OPR.mod_switch(x0.astype(np.uint64), x1.astype(np.uint64), ell, p)
        assert np.array_equal(host(y0).astype(object), np.asarray(e0, dtype=object))
        assert np.array_equal(host(y1).astype(object), np.asarray(e1, dtype=object))


def _prime_above(ell):
    import sympy
    return int(sympy.prevprime(1 << (ell + 1)))


def test_streaming_unaligned_views_and_inplace(B):
    rng = np.random.default_rng(9)
    n = 10001
    x0, x1 = rand_ring(rng, n + 1, 64), rand_ring(rng, n + 1, 64)
    d0, d1 = dev(x0), dev(x1)
    y0, y1 = B.trunc_det(d0[1:], d1[1:], 64, 13, 0)               # 8-byte, not 16-byte aligned
    e0, e1 = OPR.trunc_det(x0[1:], x1[1:], 64, 13, 0)
    assert np.array_equal(host(y0), e0) and np.array_equal(host(y1), e1)
    z0, z1 = d0.clone(), d1.clone()
    B.trunc_prob(z0, z1, 64, 13, out=(z0, z1))                     # in place
    e0, e1 = OPR.trunc_prob(x0, x1, 64, 13)
    assert np.array_equal(host(z0), e0) and np.array_equal(host(z1), e1)


def test_zero_length_is_noop(B):
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    y0, y1 = B.trunc_det(e, e, 64, 13)
    assert y0.numel() == 0
    y0, y1 = B.drelu(e, e, B.Params(64, 7, 11), B.Seeds(1, 2, 3))
    assert y0.numel() == 0


# ------------------------------------------------------------- DReLU / ReLU

# (ell, lx, k_lo): every window-count bucket of both storage widths
DRELU_CASES = [(64, 7, 11), (64, 7, 0), (64, 11, 13), (64, 15, 10), (64, 18, 13), (64, 22, 5), (64, 27, 0),
               (64, 31, 0), (64, 32, 0), (51, 11, 13), (40, 19, 2), (33, 16, 1),
               (32, 8, 8), (24, 7, 10), (32, 15, 2), (32, 16, 0), (16, 5, 3), (8, 3, 1)]


def _inputs(rng, n, ell, lx, k_lo):
    """Half inside the guard domain, a band near zero, the rest arbitrary ring elements."""
    bound = 1 << (k_lo + lx - 1)
    xs = rng.integers(-bound + 1, bound, size=n)
    x = np.array([v % (1 << ell) for v in xs.tolist()], dtype=np.uint64)
    x[: n // 8] = np.array([v % (1 << ell) for v in rng.integers(-(1 << k_lo) - 2, (1 << k_lo) + 3, size=n // 8).tolist()],
                           dtype=np.uint64)
    arb = rand_ring(rng, n, ell).astype(np.uint64)
    x[n // 2:] = arb[n // 2:]
    x[0] = 0
    R = rand_ring(rng, n, ell).astype(np.uint64)
    m = np.uint64((1 << ell) - 1) if ell < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    x0 = (x + R) & m
    x1 = ((~R) + np.uint64(1)) & m
    dt = W.storage_dtype(ell)
    return x0.astype(dt), x1.astype(dt)


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx,k_lo", DRELU_CASES)
def test_drelu_relu_parity_with_capture(B, op, ell, lx, k_lo):
    rng = np.random.default_rng(ell * 1000 + lx * 10 + k_lo)
    p = default_prime(lx)
    seeds = (0x9E3779B97F4A7C15 + lx, 0xC2B2AE3D27D4EB4F + ell, 0x165667B19E3779F9 + k_lo)
    nonce = 0xFEEDFACECAFEBEEF ^ (ell << 8)
    prm, sd = B.Params(ell, lx, k_lo), B.Seeds(*seeds, nonce)
    for n, elem_base in [(1, 0), (257, 3), (3001, (1 << 32) - 1500)]:
        x0, x1 = _inputs(rng, n, ell, lx, k_lo)
        fn = B.drelu if op == "drelu" else B.relu
        y0, y1, cap = fn(dev(x0), dev(x1), prm, sd, elem_base=elem_base, capture=True)
        ofn = OPR.drelu if op == "drelu" else OPR.relu
        e0, e1, w0, w1 = ofn(x0.astype(np.uint64), x1.astype(np.uint64), ell, lx, k_lo, p, seeds, nonce,
                             elem_base=elem_base)
        assert np.array_equal(host(y0).astype(np.uint64), e0), (n, elem_base)
        assert np.array_equal(host(y1).astype(np.uint64), e1), (n, elem_base)
        c = host(cap).astype(object).reshape(2, n, lx + 1)
        assert np.array_equal(c[0], np.asarray(w0, dtype=object)), "P0 messages"
        assert np.array_equal(c[1], np.asarray(w1, dtype=object)), "P1 messages"
        # the same call without capture gives the same outputs
        z0, z1 = fn(dev(x0), dev(x1), prm, sd, elem_base=elem_base)
        assert same(z0, y0) and same(z1, y1)


# Every window count N = l_x + 1 of both storage widths: each N is a kernel
# instance of its own (N = 2..33 at l > 32, 2..17 at l <= 32), with the
# default prime's field arithmetic.
EVERY_N = [(64, lx) for lx in range(1, 33)] + [(32, lx) for lx in range(1, 17)]


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx", EVERY_N)
def test_every_window_count(B, op, ell, lx):
    """Each instance against the oracle, bit-exact: the capturing kernel
    (outputs and round-1 messages), the production kernel (one lane per
    element, no capture: n = 20,000 gives every SIMD a wave) and the
    lane-group kernel of small calls."""
    k_lo = min(13 if ell == 64 else 8, ell - 2 * lx)
    rng = np.random.default_rng(7919 * ell + lx)
    p = default_prime(lx)
    seeds = (0x0123456789ABCDEF ^ lx, 0xFEDCBA9876543210 ^ ell, 0x5555AAAA3333CCCC + lx)
    nonce = 0xC0DE0000 + 64 * ell + lx
    prm, sd = B.Params(ell, lx, k_lo), B.Seeds(*seeds, nonce)
    fn = B.drelu if op == "drelu" else B.relu
    ofn = OPR.drelu if op == "drelu" else OPR.relu
    for n, elem_base, capture in [(1500, (1 << 32) - 700, True), (20000, 77, False), (600, 5, False)]:
        x0, x1 = _inputs(rng, n, ell, lx, k_lo)
        out = fn(dev(x0), dev(x1), prm, sd, elem_base=elem_base, capture=capture)
        e0, e1, w0, w1 = ofn(x0.astype(np.uint64), x1.astype(np.uint64), ell, lx, k_lo, p, seeds, nonce,
                             elem_base=elem_base)
        assert np.array_equal(host(out[0]).astype(np.uint64), e0), (n, "y0")
        assert np.array_equal(host(out[1]).astype(np.uint64), e1), (n, "y1")
        if capture:
            c = host(out[2]).astype(object).reshape(2, n, lx + 1)
            assert np.array_equal(c[0], np.asarray(w0, dtype=object)), "P0 messages"
            assert np.array_equal(c[1], np.asarray(w1, dtype=object)), "P1 messages"


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx", [c for c in EVERY_N if c[1] >= 2])
def test_every_window_count_explicit_prime(B, op, ell, lx):
    """The same with the next prime below the default one (the generic field
    arithmetic: fp32 quotient, fp64 quotient, Barrett or the 128-bit product,
    by the size of p): capturing and production kernels against the oracle."""
    import sympy
    p = int(sympy.prevprime(default_prime(lx)))
    assert p > (1 << lx)
    k_lo = min(13 if ell == 64 else 8, ell - 2 * lx)
    rng = np.random.default_rng(104729 * ell + lx)
    seeds = (lx, ell, 0xABCDEF)
    prm, sd = B.Params(ell, lx, k_lo, p), B.Seeds(*seeds, 99)
    fn = B.drelu if op == "drelu" else B.relu
    ofn = OPR.drelu if op == "drelu" else OPR.relu
    for n, capture in [(800, True), (20000, False)]:
        x0, x1 = _inputs(rng, n, ell, lx, k_lo)
        out = fn(dev(x0), dev(x1), prm, sd, elem_base=n, capture=capture)
        e0, e1, w0, w1 = ofn(x0.astype(np.uint64), x1.astype(np.uint64), ell, lx, k_lo, p, seeds, 99, elem_base=n)
        assert np.array_equal(host(out[0]).astype(np.uint64), e0) and np.array_equal(host(out[1]).astype(np.uint64), e1)
        if capture:
            c = host(out[2]).astype(object).reshape(2, n, lx + 1)
            assert np.array_equal(c[0], np.asarray(w0, dtype=object)) and np.array_equal(c[1], np.asarray(w1, dtype=object))


def test_drelu_explicit_prime_and_inplace(B):
    rng = np.random.default_rng(77)
    ell, lx, k_lo, p = 64, 18, 13, 524269          # a non-Mersenne prime in (2^18, 2^19)
    import sympy
    assert sympy.isprime(p)
    n = 5000
    x0, x1 = _inputs(rng, n, ell, lx, k_lo)
    seeds = (11, 22, 33)
    d0, d1 = dev(x0), dev(x1)
    y0, y1 = B.drelu(d0, d1, B.Params(ell, lx, k_lo, p), B.Seeds(*seeds, 44), out=(d0, d1))
    e0, e1, _, _ = OPR.drelu(x0, x1, ell, lx, k_lo, p, seeds, 44)
    assert np.array_equal(host(d0), e0) and np.array_equal(host(d1), e1)


def test_drelu_semantics_on_gpu(B):
    """Reconstructed GPU DReLU equals the sign bit outside the key-bit band (guard domain)."""
    rng = np.random.default_rng(5)
    ell, lx, k_lo = 64, 18, 13
    n = 200000
    xi = W.keybit_values(rng, n)
    x = W.encode(xi, 64)
    x0, x1 = W.share(x, 64, rng)
    y0, y1 = B.drelu(dev(x0), dev(x1), B.Params(ell, lx, k_lo), B.Seeds(1, 2, 3, 4))
    y = host(y0) + host(y1)
    outside = np.abs(xi) >= (1 << k_lo)
    assert np.array_equal(y[outside], (xi[outside] > 0).astype(np.uint64))
    r0, r1 = B.relu(dev(x0), dev(x1), B.Params(ell, lx, k_lo), B.Seeds(1, 2, 3, 4))
    r = host(r0) + host(r1)
    assert np.array_equal(r, x * y)


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell_in,k1,lx,k_lo", [(64, 13, 11, 13), (64, 13, 18, 13), (32, 8, 7, 10), (64, 20, 7, 11),
                                                  (64, 13, 11, 0), (32, 8, 12, 0)])
def test_fused_trunc_then_drelu_relu(B, op, ell_in, k1, lx, k_lo):
    """Alg. 5 by k1 bits fused with Alg. 7/8 equals trunc_det followed by the op, and the oracle."""
    rng = np.random.default_rng(ell_in + k1 + lx)
    ell = ell_in - k1
    n = 5003
    bound = 1 << (k_lo + lx - 1 + k1)
    xs = rng.integers(-bound + 1, bound, size=n)
    x = np.array([v % (1 << ell_in) for v in xs.tolist()], dtype=np.uint64)
    x0, x1 = W.share(x, ell_in, rng)
    seeds = (3, 1, 4)
    prm, sd = B.Params(ell, lx, k_lo), B.Seeds(*seeds, 15)
    fused = (B.trunc_relu if op == "relu" else B.trunc_drelu)(dev(x0), dev(x1), ell_in, k1, prm, sd, elem_base=9,
                                                             capture=True)
    t0, t1 = B.trunc_det(dev(x0), dev(x1), ell_in, k1)
    two = (B.relu if op == "relu" else B.drelu)(t0, t1, prm, sd, elem_base=9, capture=True)
    for a, b in zip(fused, two):
        assert same(a, b)
    e0, e1 = OPR.trunc_det(x0.astype(np.uint64), x1.astype(np.uint64), ell_in, k1)
    o0, o1, w0, w1 = (OPR.relu if op == "relu" else OPR.drelu)(e0, e1, ell, lx, k_lo, default_prime(lx), seeds, 15,
                                                               elem_base=9)
    assert np.array_equal(host(fused[0]).astype(np.uint64), o0) and np.array_equal(host(fused[1]).astype(np.uint64), o1)


def test_fused_trunc_rejects_mismatched_rings(B):
    x = torch.zeros(10, dtype=torch.int64, device="cuda")
    with pytest.raises(B.BicopError):
        B.trunc_relu(x, x, 64, 13, B.Params(50, 11, 13), B.Seeds(1, 2, 3))        # 64 - 13 != 50
    with pytest.raises(B.BicopError):
        B.trunc_relu(x, x, 40, 10, B.Params(30, 7, 10), B.Seeds(1, 2, 3))         # 8-byte in, 4-byte out


@pytest.mark.parametrize("ell,lx,k_lo", [(64, 18, 13), (64, 32, 0), (64, 31, 0), (64, 7, 11), (51, 11, 13),
                                         (32, 8, 8), (24, 7, 10), (64, 2, 5), (64, 16, 13), (64, 21, 13),
                                         (64, 23, 13), (64, 24, 13), (64, 27, 5)])
def test_lane_groups_agree_with_one_lane(B, ell, lx, k_lo):
    """Small calls spread each element over 4 or 8 lanes (mask blocks split
    among the lanes, or for the mask bit stream drawn by the lanes into LDS
    and read back per slot; P2's minimum combined by lane shuffles).  Forcing
    each group size through the schedule table gives identical outputs, for
    the stream's shifted (N = 17..24), 32-bit (N = 25..32) and 64-bit (N = 33)
    fields alike, and for element indices across 2^32."""
    rng = np.random.default_rng(ell + 100 * lx + k_lo)
    prm = B.Params(ell, lx, k_lo)
    w = B.ring_width(ell)
    before = {o: B.get_schedule("group", lx + 1, w, o) for o in (B.BC_OP_DRELU, B.BC_OP_RELU)}
    try:
        for n, elem_base in [(1, 0), (5, 7), (999, (1 << 32) - 400), (12000, 12345)]:
            x0, x1 = _inputs(rng, n, ell, lx, k_lo)
            sd = B.Seeds(11, 22, 33, n)
            for fn in (B.drelu, B.relu):
                outs = []
                for gmax in (1, 4, 8):
                    B.set_schedule("group", lx + 1, gmax, w)
                    outs.append(fn(dev(x0), dev(x1), prm, sd, elem_base=elem_base))
                for o in outs[1:]:
                    assert same(o[0], outs[0][0]) and same(o[1], outs[0][1]), (fn.__name__, n)
    finally:
        for o, v in before.items():
            B.set_schedule("group", lx + 1, v, w, o)


def test_lane_groups_fused_truncation(B):
    """bc_trunc_relu on small calls (lane groups) equals the two passes."""
    rng = np.random.default_rng(91)
    prm = B.Params(51, 11, 13)
    for n in (3, 700, 30000):
        x0 = rand_ring(rng, n, 64)
        x1 = rand_ring(rng, n, 64)
        sd = B.Seeds(5, 6, 7, n)
        f0, f1 = B.trunc_relu(dev(x0), dev(x1), 64, 13, prm, sd)
        t0, t1 = B.trunc_det(dev(x0), dev(x1), 64, 13)
        r0, r1 = B.relu(t0, t1, prm, sd)
        assert same(f0, r0) and same(f1, r1)


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx,k_lo", [(64, 18, 13), (32, 8, 8)])
def test_narrow_grid_many_elements_per_thread(B, op, ell, lx, k_lo):
    """The one-call kernel on one block per compute unit: each thread walks
    three or four elements, loading each element's shares one element ahead,
    and the last stride is ragged.  Every element against the oracle (Alg. 7 /
    Alg. 8), and the same with the tuned grid."""
    rng = np.random.default_rng(4242 + lx)
    p = default_prime(lx)
    seeds = (0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0 + lx)
    nonce = 0x5EED + lx
    prm, sd = B.Params(ell, lx, k_lo), B.Seeds(*seeds, nonce)
    w = B.ring_width(ell)
    code = B.BC_OP_RELU if op == "relu" else B.BC_OP_DRELU
    fn = B.relu if op == "relu" else B.drelu
    n = 3 * 256 * 256 + 1001
    x0, x1 = _inputs(rng, n, ell, lx, k_lo)
    before = B.get_schedule("fused", lx + 1, w, code)
    try:
        B.set_schedule("fused", lx + 1, 1, w, code)
        y0, y1 = fn(dev(x0), dev(x1), prm, sd, elem_base=3)
    finally:
        B.set_schedule("fused", lx + 1, before, w, code)
    ofn = OPR.drelu if op == "drelu" else OPR.relu
    e0, e1, _, _ = ofn(x0.astype(np.uint64), x1.astype(np.uint64), ell, lx, k_lo, p, seeds, nonce, elem_base=3)
    assert np.array_equal(host(y0).astype(np.uint64), e0)
    assert np.array_equal(host(y1).astype(np.uint64), e1)
    z0, z1 = fn(dev(x0), dev(x1), prm, sd, elem_base=3)
    assert same(z0, y0) and same(z1, y1)
