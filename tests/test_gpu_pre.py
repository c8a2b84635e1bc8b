"""Precomputed randomness: the offline expansion plus the online kernel give
exactly the outputs and round-1 messages of the fused kernel (and so of the
oracle), for every field type."""

import numpy as np
import pytest

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
    return torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()


def host(t):
    t = t.detach().cpu()
    return t.view(torch.int64).numpy().view(np.uint64) if t.element_size() == 8 else \
        t.view(torch.int32).numpy().view(np.uint32)


def same(a, b):
    """Bitwise equality of two integer tensors of the same element size."""
    def v(t):
        return t.view(torch.int64) if t.element_size() == 8 else t.view(torch.int32)
    return a.shape == b.shape and a.element_size() == b.element_size() and torch.equal(v(a), v(b))


CASES = [(64, 7, 11), (64, 11, 13), (64, 15, 10), (64, 16, 3), (64, 18, 13), (64, 20, 4), (64, 27, 0), (64, 31, 0),
         (64, 32, 0), (32, 8, 8), (24, 7, 10), (32, 16, 0)]


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx,k_lo", CASES)
def test_pre_equals_fused(B, op, ell, lx, k_lo):
    rng = np.random.default_rng(ell * 100 + lx)
    n = 3001
    bound = 1 << (k_lo + lx - 1)
    x = np.array([v % (1 << ell) for v in rng.integers(-bound + 1, bound, size=n).tolist()], dtype=np.uint64)
    x0, x1 = W.share(x, ell, rng)
    d0, d1 = dev(x0), dev(x1)
    prm = B.Params(ell, lx, k_lo)
    seeds = B.Seeds(0x1111, 0x2222, 0x3333, 0x4444 + lx)
    opc = B.BC_OP_RELU if op == "relu" else B.BC_OP_DRELU
    elem_base = (1 << 33) + 5
    fused = (B.relu if op == "relu" else B.drelu)(d0, d1, prm, seeds, elem_base=elem_base, capture=True)
    rand = B.rand_expand(opc, prm, seeds, n, elem_base=elem_base)
    assert rand.numel() == B.rand_bytes(opc, prm, n)
    pre = (B.relu_pre if op == "relu" else B.drelu_pre)(d0, d1, prm, rand, capture=True)
    for a, b in zip(fused, pre):
        assert same(a, b)
    k = 200
    ofn = OPR.relu if op == "relu" else OPR.drelu
    e0, e1, w0, w1 = ofn(x0[:k].astype(np.uint64), x1[:k].astype(np.uint64), ell, lx, k_lo, default_prime(lx),
                         (0x1111, 0x2222, 0x3333), 0x4444 + lx, elem_base=elem_base)
    assert np.array_equal(host(pre[0])[:k].astype(np.uint64), e0)
    assert np.array_equal(host(pre[1])[:k].astype(np.uint64), e1)
    cap = host(pre[2]).astype(object).reshape(2, n, lx + 1)
    assert np.array_equal(cap[0, :k], np.asarray(w0, dtype=object))
    assert np.array_equal(cap[1, :k], np.asarray(w1, dtype=object))


def test_pre_rejects_small_buffer(B):
    prm = B.Params(64, 7, 11)
    small = torch.empty(B.rand_bytes(B.BC_OP_RELU, prm, 100) - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BicopError) as ei:
        B.rand_expand(B.BC_OP_RELU, prm, B.Seeds(1, 2, 3), 100, out=small)
    assert ei.value.code == -7
    x = torch.zeros(100, dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):                      # a buffer bc_rand_expand did not describe
        B.relu_pre(x, x, prm, small)


def test_pre_refuses_a_record_of_another_call(B):
    """A record read with another op, setting, length, nonce or element offset
    is refused on the host with BC_ERR_ARG (its description says what it was
    expanded for); nothing is launched and the outputs stay as they were."""
    prm = B.Params(64, 7, 11)
    rec = B.rand_expand(B.BC_OP_RELU, prm, B.Seeds(1, 2, 3, 4), 100)
    x = torch.ones(100, dtype=torch.int64, device="cuda")
    y = (torch.full_like(x, 7), torch.full_like(x, 7))
    cases = [(B.relu_pre, x[:99], prm, {}), (B.drelu_pre, x, prm, {}), (B.relu_pre, x, B.Params(64, 7, 10), {}),
             (B.relu_pre, x, B.Params(64, 8, 11), {}), (B.relu_pre, x, B.Params(51, 7, 11), {}),
             (B.relu_pre, x, prm, {"seeds": B.Seeds(1, 2, 3, 5)}), (B.relu_pre, x, prm, {"elem_base": 7})]
    for fn, xs, p, kw in cases:
        with pytest.raises(B.BicopError) as ei:
            fn(xs, xs, p, rec, out=(y[0][:xs.numel()], y[1][:xs.numel()]), **kw)
        assert ei.value.code == -8, (fn.__name__, xs.numel(), p, kw)
    torch.cuda.synchronize()
    assert bool((y[0] == 7).all()) and bool((y[1] == 7).all())
    z0, z1 = B.relu_pre(x, x, prm, rec)                  # the matching call runs
    assert z0.numel() == 100


PACKING_CASES = [(64, 3, 5), (64, 4, 5), (64, 5, 5), (64, 6, 5), (64, 9, 5), (64, 10, 5), (64, 12, 5), (64, 21, 5),
                 (64, 24, 5), (64, 25, 5), (32, 3, 2), (32, 5, 4), (20, 6, 3)]


@pytest.mark.parametrize("op", ["drelu", "relu"])
@pytest.mark.parametrize("ell,lx,k_lo", PACKING_CASES)
def test_pre_record_packing_against_oracle(B, op, ell, lx, k_lo):
    """Window counts N = l_x + 1 whose 2N draws fill the record's N-bit
    fields (floor(64 / N) per word) exactly, or leave a partial last word:
    every output and every captured message against the oracle, for n from
    one element to a ragged block."""
    rng = np.random.default_rng(7 * ell + lx)
    prm = B.Params(ell, lx, k_lo)
    seeds = B.Seeds(0x5151, 0x6262, 0x7373, 0x8484 + lx)
    opc = B.BC_OP_RELU if op == "relu" else B.BC_OP_DRELU
    ofn = OPR.relu if op == "relu" else OPR.drelu
    bound = 1 << (k_lo + lx - 1)
    for n in (1, 2, 63, 300):
        print(f"pre packing op={op} ell={ell} lx={lx} k_lo={k_lo} n={n}", flush=True)
        x = np.array([v % (1 << ell) for v in rng.integers(-bound + 1, bound, size=n).tolist()], dtype=np.uint64)
        x0, x1 = W.share(x, ell, rng)
        rand = B.rand_expand(opc, prm, seeds, n, elem_base=17)
        y0, y1, cap = (B.relu_pre if op == "relu" else B.drelu_pre)(dev(x0), dev(x1), prm, rand, capture=True)
        e0, e1, w0, w1 = ofn(x0.astype(np.uint64), x1.astype(np.uint64), ell, lx, k_lo, default_prime(lx),
                             (0x5151, 0x6262, 0x7373), 0x8484 + lx, elem_base=17)
        assert np.array_equal(host(y0).astype(np.uint64), e0)
        assert np.array_equal(host(y1).astype(np.uint64), e1)
        c = host(cap).astype(object).reshape(2, n, lx + 1)
        assert np.array_equal(c[0], np.asarray(w0, dtype=object))
        assert np.array_equal(c[1], np.asarray(w1, dtype=object))
