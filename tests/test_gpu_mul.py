"""GPU parity of the elementwise product with truncation (Alg. linear,
truncate-then-multiply, and multiply-then-truncate) through the C ABI
against the CPU oracle, bit-exact (tolerance 0).

Rings of both storage widths, odd and even f, all three orders; sizes
from one element to several blocks with a ragged tail, unaligned views
(the scalar path), element indices across 2^32, in place, zero length.
At the bench's size: samples against the oracle and the e1 counts of both
orders against their expected rates.
"""

import numpy as np
import pytest

from oracle import protocols as OPR
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = np.uint64
SEEDS = (0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0)


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


def rand_ring(rng, n, ell):
    v = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * U64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    if ell < 64:
        v &= U64((1 << ell) - 1)
    return v.astype(W.storage_dtype(ell))


CASES = [(64, 26), (64, 13), (64, 1), (64, 63), (51, 13), (40, 7), (33, 10), (32, 8), (32, 13), (24, 5), (8, 3),
         (1, 0)]
ORDERS = {"before": 2, "after": 1, "none": 0}


@pytest.mark.parametrize("order", list(ORDERS))
@pytest.mark.parametrize("ell,f", CASES)
def test_mul_trunc_parity(B, order, ell, f):
    code = ORDERS[order]
    if code == 0:
        f = 0
    if code == 1 and f >= ell:
        pytest.skip("f >= ell")
    rng = np.random.default_rng(ell * 100 + f + 7 * code)
    nonce = 0xC0DE + ell
    for n, elem_base in [(1, 0), (3, 5), (257, 11), (4097, (1 << 32) - 2000), (65537, 123)]:
        print(f"mul {order} ell={ell} f={f} n={n} base={elem_base}", flush=True)
        x0, x1, y0, y1 = (rand_ring(rng, n, ell) for _ in range(4))
        z0, z1 = B.mul_trunc(dev(x0), dev(x1), dev(y0), dev(y1), ell, f, code, B.Seeds(*SEEDS, nonce),
                             elem_base=elem_base)
        e0, e1 = OPR.mul_trunc(*(v.astype(U64) for v in (x0, x1, y0, y1)), ell, f, code, SEEDS, nonce,
                               elem_base=elem_base)
        assert np.array_equal(host(z0).astype(U64), e0), (n, elem_base)
        assert np.array_equal(host(z1).astype(U64), e1), (n, elem_base)


def test_mul_trunc_unaligned_views_and_inplace(B):
    rng = np.random.default_rng(3)
    ell, f, n = 64, 26, 10001
    x0, x1, y0, y1 = (rand_ring(rng, n + 1, ell) for _ in range(4))
    d = [dev(v) for v in (x0, x1, y0, y1)]
    views = [t[1:] for t in d]                          # 8 bytes past a 16-byte boundary: the scalar path
    z0, z1 = B.mul_trunc(*views, ell, f, B.BC_TRUNC_BEFORE, B.Seeds(*SEEDS, 9))
    e0, e1 = OPR.mul_trunc(x0[1:], x1[1:], y0[1:], y1[1:], ell, f, OPR.TRUNC_BEFORE, SEEDS, 9)
    assert np.array_equal(host(z0), e0) and np.array_equal(host(z1), e1)
    # in place over x
    B.mul_trunc(d[0], d[1], d[2], d[3], ell, f, B.BC_TRUNC_AFTER, B.Seeds(*SEEDS, 9), out=(d[0], d[1]))
    e0, e1 = OPR.mul_trunc(x0, x1, y0, y1, ell, f, OPR.TRUNC_AFTER, SEEDS, 9)
    assert np.array_equal(host(d[0]), e0) and np.array_equal(host(d[1]), e1)


def test_mul_trunc_zero_length(B):
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    z0, z1 = B.mul_trunc(e, e, e, e, 64, 26, B.BC_TRUNC_BEFORE, B.Seeds(*SEEDS))
    assert z0.numel() == 0 and z1.numel() == 0


def test_e1_counts_at_2p24(B):
    """The bench's workload: 2^24 pairs of 31-bit fixed-point values (5 integer
    and 26 fractional bits) in Z_2^64.  Multiply-then-truncate fails (|error| >
    1) at the rate mean(|x y|) / 2^64; truncate-then-multiply never does and
    stays within the precision it gives up.  Samples match the oracle."""
    (x, (x0, x1)), (y, (y0, y1)) = W.linear_factors(seed=5)
    n = x.size
    d = [dev(v) for v in (x0, x1, y0, y1)]
    sd = B.Seeds(*SEEDS, 77)
    za = B.mul_trunc(*d, 64, 26, B.BC_TRUNC_AFTER, sd)
    zb = B.mul_trunc(*d, 64, 26, B.BC_TRUNC_BEFORE, sd)
    xs, ys = W.signed_values(x, 64).astype(np.int64), W.signed_values(y, 64).astype(np.int64)
    exact = (xs * ys) >> 26                                    # |x y| < 2^62: exact in int64
    ra = (host(za[0]) + host(za[1])).view(np.int64)
    rb = (host(zb[0]) + host(zb[1])).view(np.int64)
    fails_a = int(np.count_nonzero(np.abs(ra - exact) > 1))
    rate = float(np.mean(np.abs(xs.astype(np.float64) * ys.astype(np.float64)))) / 2.0 ** 64
    assert abs(fails_a - rate * n) < 6 * np.sqrt(rate * n)
    err_b = np.abs(rb - exact)
    assert int(err_b.max()) < (1 << 19)
    idx = np.unique(np.concatenate([np.arange(200), np.arange(n - 200, n),
                                    np.random.default_rng(1).integers(0, n, size=2000)]))
    for z, code in ((za, OPR.TRUNC_AFTER), (zb, OPR.TRUNC_BEFORE)):
        e0, e1 = OPR.mul_trunc(x0[idx], x1[idx], y0[idx], y1[idx], 64, 26, code, SEEDS, 77, g=idx.astype(U64))
        assert np.array_equal(host(z[0])[idx], e0) and np.array_equal(host(z[1])[idx], e1)
