"""GPU parity of the DReLU with the parties apart (bc_drelu_send, bc_drelu_reply,
bc_drelu_finish) through the C ABI against the CPU oracle, bit-exact: every
packed message word, every reply share and every output.  The unpacked
messages equal bc_drelu's captured ones and send -> reply -> finish equals
the fused bc_drelu, up to the bench's 2^24 key-bit elements.
"""

import numpy as np
import pytest

from oracle import protocols as OPR
from oracle.params import default_prime
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = np.uint64
SEEDS = (0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0)
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


def _shares(rng, n, ell, lx, k_lo):
    bound = 1 << (k_lo + lx - 1)
    xs = rng.integers(-bound + 1, bound, size=n)
    x = np.array([v % (1 << ell) for v in xs.tolist()], dtype=U64)
    x[0] = 0
    R = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * U64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    m = U64((1 << ell) - 1) if ell < 64 else U64(0xFFFFFFFFFFFFFFFF)
    dt = W.storage_dtype(ell)
    return ((x + R) & m).astype(dt), ((~R + U64(1)) & m).astype(dt)


@pytest.mark.parametrize("ell,lx,k_lo", CASES)
def test_split_parity(B, ell, lx, k_lo):
    rng = np.random.default_rng(ell * 100 + lx)
    p = default_prime(lx)
    prm = B.Params(ell, lx, k_lo)
    nonce = 0xABC0 + lx
    sd = B.Seeds(*SEEDS, nonce)
    for n, base in [(1, 0), (257, 9), (3001, (1 << 32) - 1000)]:
        print(f"split ell={ell} lx={lx} k_lo={k_lo} n={n} base={base}", flush=True)
        x0, x1 = _shares(rng, n, ell, lx, k_lo)
        d0_, d1_ = dev(x0), dev(x1)
        m0 = B.drelu_send(0, d0_, prm, sd, elem_base=base)
        m1 = B.drelu_send(1, d1_, prm, sd, elem_base=base)
        o0 = OPR.drelu_send(0, x0.astype(U64), ell, lx, k_lo, p, SEEDS, nonce, elem_base=base)
        o1 = OPR.drelu_send(1, x1.astype(U64), ell, lx, k_lo, p, SEEDS, nonce, elem_base=base)
        assert np.array_equal(host(m0).reshape(o0.shape), o0), "P0 words"
        assert np.array_equal(host(m1).reshape(o1.shape), o1), "P1 words"
        r0, r1 = B.drelu_reply(m0, m1, prm, sd, elem_base=base)
        e0, e1 = OPR.drelu_reply(o0, o1, ell, lx, p, SEEDS, nonce, elem_base=base)
        assert np.array_equal(host(r0).astype(U64), e0) and np.array_equal(host(r1).astype(U64), e1)
        y0 = B.drelu_finish(0, r0, prm, sd, elem_base=base)
        y1 = B.drelu_finish(1, r1, prm, sd, elem_base=base)
        f0, f1, c = B.drelu(d0_, d1_, prm, sd, elem_base=base, capture=True)
        assert torch.equal(y0, f0) and torch.equal(y1, f1)
        cap = host(c).astype(object).reshape(2, n, lx + 1)
        assert np.array_equal(OPR.unpack_messages(host(m0).reshape(o0.shape), lx + 1), cap[0])
        assert np.array_equal(OPR.unpack_messages(host(m1).reshape(o1.shape), lx + 1), cap[1])


def test_split_finish_in_place(B):
    rng = np.random.default_rng(2)
    x0, x1 = _shares(rng, 5000, 64, 7, 11)
    prm, sd = B.Params(64, 7, 11), B.Seeds(*SEEDS, 3)
    m0, m1 = B.drelu_send(0, dev(x0), prm, sd), B.drelu_send(1, dev(x1), prm, sd)
    r0, r1 = B.drelu_reply(m0, m1, prm, sd)
    B.drelu_finish(0, r0, prm, sd, out=r0)
    B.drelu_finish(1, r1, prm, sd, out=r1)
    f0, f1 = B.drelu(dev(x0), dev(x1), prm, sd)
    assert torch.equal(r0, f0) and torch.equal(r1, f1)


@pytest.mark.parametrize("lx,k_lo", [(18, 13), (7, 11)])
def test_split_equals_fused_2p24(B, lx, k_lo):
    """The bench's 2^24 key-bit values: the three parties' kernels give the
    fused call's outputs on every element; the messages match the oracle on
    samples."""
    _, (x0, x1), _, _ = W.keybit_drelu(seed=2, n=1 << 24)
    prm, sd = B.Params(64, lx, k_lo), B.Seeds(*SEEDS, 61)
    d0_, d1_ = dev(x0), dev(x1)
    m0, m1 = B.drelu_send(0, d0_, prm, sd), B.drelu_send(1, d1_, prm, sd)
    r0, r1 = B.drelu_reply(m0, m1, prm, sd)
    y0, y1 = B.drelu_finish(0, r0, prm, sd), B.drelu_finish(1, r1, prm, sd)
    f0, f1 = B.drelu(d0_, d1_, prm, sd)
    assert torch.equal(y0, f0) and torch.equal(y1, f1)
    n = x0.size
    idx = np.unique(np.concatenate([np.arange(100), np.arange(n - 100, n),
                                    np.random.default_rng(4).integers(0, n, size=500)]))
    o0 = OPR.drelu_send(0, x0[idx], 64, lx, k_lo, default_prime(lx), SEEDS, 61, g=idx.astype(U64))
    assert np.array_equal(host(m0)[:, idx], o0)


def test_split_zero_length(B):
    prm, sd = B.Params(64, 18, 13), B.Seeds(*SEEDS)
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    m0, m1 = B.drelu_send(0, e, prm, sd), B.drelu_send(1, e, prm, sd)
    assert tuple(m0.shape) == (B.msg_words(19), 0)
    r0, r1 = B.drelu_reply(m0, m1, prm, sd)
    assert r0.numel() == 0 and B.drelu_finish(0, r0, prm, sd).numel() == 0
