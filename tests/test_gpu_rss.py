"""GPU parity of the replicated-sharing DReLU / ReLU (Alg. drelu2 and the RSS
ReLU of the appendix) through the C ABI against the CPU oracle, bit-exact:
every output share and every captured round-1 message (tolerance 0).

Settings cover every window-count bucket of both storage widths; sizes span
one element, several thread blocks with a ragged tail, and element indices
across 2^32.  At larger sizes the outputs are checked against properties that
hold at any size: the DReLU reconstructs to the sign outside the key-bit band
and the ReLU to x DReLU(x).
"""

import numpy as np
import pytest

from oracle import protocols as OPR
from oracle.params import default_prime
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = np.uint64
SEEDS5 = (0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89, 0x452821E638D01377)

# (ell, lx, k_lo): every window-count bucket of both storage widths
CASES = [(64, 7, 11), (64, 7, 0), (64, 11, 13), (64, 15, 10), (64, 18, 13), (64, 22, 5), (64, 27, 0),
         (64, 31, 0), (64, 32, 0), (51, 11, 13), (40, 19, 2), (33, 16, 1),
         (32, 8, 8), (24, 7, 10), (32, 15, 2), (32, 16, 0), (16, 5, 3), (8, 3, 1)]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop
    return bicop


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int64 if a.dtype == U64 else np.int32)).cuda()


def host(t):
    t = t.detach().cpu()
    if t.element_size() == 8:
        return t.view(torch.int64).numpy().view(U64)
    return t.view(torch.int32).numpy().view(np.uint32)


def recon(ys, ell):
    s = ys[0].astype(U64) + ys[1].astype(U64) + ys[2].astype(U64)
    return s & U64((1 << ell) - 1) if ell < 64 else s


def _values(rng, n, ell, lx, k_lo):
    """Half inside the guard domain (an eighth in the key-bit band), the rest
    arbitrary ring elements, and x = 0 first."""
    bound = 1 << (k_lo + lx - 1)
    xs = rng.integers(-bound + 1, bound, size=n)
    xs[: n // 8] = rng.integers(-(1 << k_lo) - 2, (1 << k_lo) + 3, size=n // 8)
    x = np.array([v % (1 << ell) for v in xs.tolist()], dtype=U64)
    arb = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * U64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    if ell < 64:
        arb &= U64((1 << ell) - 1)
    x[n // 2:] = arb[n // 2:]
    x[0] = 0
    return x


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx,k_lo", CASES)
def test_rss_parity_with_capture(B, op, ell, lx, k_lo):
    rng = np.random.default_rng(ell * 1000 + lx * 10 + k_lo + 7)
    p = default_prime(lx)
    nonce = 0x5EED0000 + ell * 64 + lx
    sd = B.RssSeeds(SEEDS5[0], SEEDS5[1], SEEDS5[2], SEEDS5[3], SEEDS5[4], nonce)
    prm = B.Params(ell, lx, k_lo)
    fn = B.rss_drelu if op == "drelu" else B.rss_relu
    ofn = OPR.rss_drelu if op == "drelu" else OPR.rss_relu
    for n, elem_base in [(1, 0), (257, 3), (3001, (1 << 32) - 1500)]:
        print(f"rss {op} ell={ell} lx={lx} k_lo={k_lo} n={n} base={elem_base}", flush=True)
        xs = W.share3(_values(rng, n, ell, lx, k_lo), ell, rng)
        ys, cap = fn(tuple(dev(a) for a in xs), prm, sd, elem_base=elem_base, capture=True)
        e, w0, w1 = ofn(*(a.astype(U64) for a in xs), ell, lx, k_lo, p, SEEDS5, nonce, elem_base=elem_base)
        for j in range(3):
            assert np.array_equal(host(ys[j]).astype(U64), e[j]), (j, n, elem_base)
        c = host(cap).astype(object).reshape(2, n, lx + 1)
        assert np.array_equal(c[0], np.asarray(w0, dtype=object)), "P0 messages"
        assert np.array_equal(c[1], np.asarray(w1, dtype=object)), "P1 messages"
        zs = fn(tuple(dev(a) for a in xs), prm, sd, elem_base=elem_base)
        for j in range(3):
            assert torch.equal(zs[j], ys[j])


def test_rss_round1_is_the_2of2_round1(B):
    """P0 enters [x]_0 + [x]_1 and P1 enters [x]_2: the captured messages equal
    those of bc_drelu on that 2-of-2 input with the same seed_01 and nonce."""
    rng = np.random.default_rng(21)
    ell, lx, k_lo, n = 64, 18, 13, 20000
    xs = W.share3(_values(rng, n, ell, lx, k_lo), ell, rng)
    d = [dev(a) for a in xs]
    _, cap = B.rss_drelu(tuple(d), B.Params(ell, lx, k_lo), B.RssSeeds(*SEEDS5, 99), capture=True)
    _, _, cap2 = B.drelu(dev(xs[0] + xs[1]), d[2], B.Params(ell, lx, k_lo), B.Seeds(*SEEDS5[:3], 99), capture=True)
    assert torch.equal(cap, cap2)


def test_rss_explicit_prime_and_inplace(B):
    rng = np.random.default_rng(77)
    ell, lx, k_lo, p = 64, 18, 13, 524269          # a non-Mersenne prime in (2^18, 2^19)
    n = 5000
    xs = W.share3(_values(rng, n, ell, lx, k_lo), ell, rng)
    for fn, ofn in ((B.rss_drelu, OPR.rss_drelu), (B.rss_relu, OPR.rss_relu)):
        d = tuple(dev(a) for a in xs)
        fn(d, B.Params(ell, lx, k_lo, p), B.RssSeeds(*SEEDS5, 44), out=d)
        e, _, _ = ofn(*xs, ell, lx, k_lo, p, SEEDS5, 44)
        for j in range(3):
            assert np.array_equal(host(d[j]), e[j])


def test_rss_zero_length(B):
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    ys = B.rss_relu((e, e, e), B.Params(64, 7, 11), B.RssSeeds(*SEEDS5))
    assert all(y.numel() == 0 for y in ys)


@pytest.mark.parametrize("ell,lx,k_lo,n", [(64, 18, 13, 1 << 20), (64, 7, 11, 1 << 20), (32, 8, 8, 300001)])
def test_rss_properties_at_size(B, ell, lx, k_lo, n):
    """Guard-domain values: DReLU = [x > 0] outside the band |x| < 2^k_lo and a
    bit inside it; ReLU = x DReLU(x) everywhere; the oracle on samples."""
    rng = np.random.default_rng(n + lx)
    bound = 1 << (k_lo + lx - 1)
    xi = rng.integers(-bound + 1, bound, size=n)
    x = W.encode(xi, ell).astype(U64)
    xs = W.share3(x, ell, rng)
    d = tuple(dev(a) for a in xs)
    prm, sd = B.Params(ell, lx, k_lo), B.RssSeeds(*SEEDS5, 1234)
    yd = [host(t).astype(U64) for t in B.rss_drelu(d, prm, sd)]
    yr = [host(t).astype(U64) for t in B.rss_relu(d, prm, sd)]
    dr, rr = recon(yd, ell), recon(yr, ell)
    assert np.all((dr == 0) | (dr == 1))
    outside = np.abs(xi) >= (1 << k_lo)
    assert np.array_equal(dr[outside], (xi[outside] > 0).astype(U64))
    m = U64((1 << ell) - 1) if ell < 64 else U64(0xFFFFFFFFFFFFFFFF)
    assert np.array_equal(rr, (x * dr) & m)
    idx = np.unique(np.concatenate([np.arange(300), np.arange(n - 300, n), rng.integers(0, n, size=2000)]))
    e, _, _ = OPR.rss_relu(*(a[idx].astype(U64) for a in xs), ell, lx, k_lo, default_prime(lx), SEEDS5, 1234,
                           g=idx.astype(U64))
    for j in range(3):
        assert np.array_equal(yr[j][idx], e[j])
