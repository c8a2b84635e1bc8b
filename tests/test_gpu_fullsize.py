"""GPU parity at the workloads' full sizes, in the launch configuration that
bench.py times (the binding applies the same autotuned schedule table).

* Streaming outputs (trunc_det) are compared with the oracle on every element.
* DReLU / ReLU outputs are compared with the oracle, bit-exact, on every
  element of the 65,536-element plain calls, of the 2^24-element key-bit
  DReLU and ReLU, and of the largest ResNet-18 tensor (25,690,112 elements)
  in the ragged batch and in the layer chain; the oracle runs over chunks of
  elements in the session's forked worker processes (tests/oracle_pool.py).
  The other segments are compared on sampled element indices: the oracle
  draws each element's randomness from its global index, so any element can
  be recomputed on its own.
* Every element is also checked against properties that hold at any size
  (Alg. 7 and 8 with the key-bit window, Sec. 6.1):
    - a DReLU output reconstructs to 0 or 1, and to [x > 0] wherever
      |x| >= 2^k_lo (outside the key-bit band);
    - a ReLU output reconstructs to 0 or x, and to x [x > 0] outside the band.
"""

import numpy as np
import pytest

from oracle import protocols as OPR
from oracle.params import default_prime
from oracle_pool import protocol_all
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


def recon(y0, y1, ell):
    s = y0.astype(U64) + y1.astype(U64)
    return s & U64((1 << ell) - 1) if ell < 64 else s


def signed(x, ell):
    return W.signed_values(np.asarray(x).astype(U64), ell)


def sample_indices(n, rng, k=3000):
    idx = np.concatenate([np.arange(min(n, 500)), np.arange(max(0, n - 500), n), rng.integers(0, n, size=k)])
    return np.unique(idx)


def check_drelu_property(y, xi, k_lo):
    assert np.all((y == 0) | (y == 1))
    outside = np.abs(xi) >= (1 << k_lo)
    assert np.array_equal(y[outside], (xi[outside] > 0).astype(U64))


def check_relu_property(y, x, xi, k_lo):
    assert np.all((y == 0) | (y == x))
    outside = np.abs(xi) >= (1 << k_lo)
    want = np.where(xi[outside] > 0, x[outside], U64(0))
    assert np.array_equal(y[outside], want)


@pytest.mark.parametrize("lx", [32, 31])
def test_plain_drelu_relu_65536_every_element(B, lx):
    """Plain DReLU / ReLU: 65,536 elements, l = 64, no key-bit reduction."""
    x, (x0, x1) = W.plain_drelu(seed=1)
    prm, nonce = B.Params(64, lx, 0), 11
    d0, d1 = dev(x0), dev(x1)
    p = default_prime(lx)
    for fn, ofn in ((B.drelu, OPR.drelu), (B.relu, OPR.relu)):
        y0, y1 = fn(d0, d1, prm, B.Seeds(*SEEDS, nonce))
        o0, o1, _, _ = ofn(x0, x1, 64, lx, 0, p, SEEDS, nonce)
        assert np.array_equal(host(y0), o0) and np.array_equal(host(y1), o1)


def test_keybit_step_2p24(B, oracle_pool):
    """The bench step: trunc_det(13) of 2^24 products and the key-bit DReLU of
    2^24 values, in the production kernel (one lane per element, no capture),
    against the oracle on every element; the sign property on every element."""
    x, (x0, x1), z, (z0, z1) = W.keybit_drelu(seed=2, n=1 << 24)
    n = x.size
    t0, t1 = B.trunc_det(dev(z0), dev(z1), 64, 13, 0)
    e0, e1 = OPR.trunc_det(z0, z1, 64, 13, 0)
    assert np.array_equal(host(t0), e0) and np.array_equal(host(t1), e1)
    del t0, t1, e0, e1

    prm, nonce = B.Params(64, 18, 13), 7
    g0, g1 = B.drelu(dev(x0), dev(x1), prm, B.Seeds(*SEEDS, nonce))
    y0, y1 = host(g0), host(g1)
    check_drelu_property(recon(y0, y1, 64), signed(x, 64), 13)
    o0, o1 = protocol_all(oracle_pool, "drelu", x0, x1, 64, 18, 13, (1 << 19) - 1, SEEDS, nonce)
    assert np.array_equal(y0, o0) and np.array_equal(y1, o1)


def test_keybit_relu_2p24(B, oracle_pool):
    """The key-bit ReLU (Alg. 8) of the same 2^24 values: the oracle on every
    element, and x DReLU(x) with the sign property on every element."""
    x, (x0, x1), _, _ = W.keybit_drelu(seed=2, n=1 << 24)
    prm, nonce = B.Params(64, 18, 13), 8
    g0, g1 = B.relu(dev(x0), dev(x1), prm, B.Seeds(*SEEDS, nonce))
    y0, y1 = host(g0), host(g1)
    check_relu_property(recon(y0, y1, 64), x, signed(x, 64), 13)
    o0, o1 = protocol_all(oracle_pool, "relu", x0, x1, 64, 18, 13, (1 << 19) - 1, SEEDS, nonce)
    assert np.array_equal(y0, o0) and np.array_equal(y1, o1)


@pytest.mark.parametrize("ell,k1,lx,k_lo", [(64, 13, 11, 13), (32, 8, 7, 10)])
def test_matmul_relu_4m_outputs(B, ell, k1, lx, k_lo):
    """ReLU after the [4096 x 4096].[4096 x 1024] fixed-point product: the
    fused truncate-then-ReLU equals the two passes on every output, the
    property holds on every output, and samples match the oracle."""
    z, (z0, z1) = W.matmul_relu(seed=3, ell=ell)
    n = z.size
    ell_out = ell - k1
    prm, nonce = B.Params(ell_out, lx, k_lo), 9
    sd = B.Seeds(*SEEDS, nonce)
    d0, d1 = dev(z0), dev(z1)
    f0, f1 = B.trunc_relu(d0, d1, ell, k1, prm, sd)
    t0, t1 = B.trunc_det(d0, d1, ell, k1, 0)
    r0, r1 = B.relu(t0, t1, prm, sd)
    assert torch.equal(f0, r0) and torch.equal(f1, r1)
    e0, e1 = OPR.trunc_det(z0.astype(U64), z1.astype(U64), ell, k1, 0)
    assert np.array_equal(host(t0).astype(U64), e0) and np.array_equal(host(t1).astype(U64), e1)
    xt = recon(e0, e1, ell_out)
    y0, y1 = host(f0).astype(U64), host(f1).astype(U64)
    check_relu_property(recon(y0, y1, ell_out), xt, signed(xt, ell_out), k_lo)
    idx = sample_indices(n, np.random.default_rng(6))
    o0, o1, _, _ = OPR.relu(e0[idx], e1[idx], ell_out, lx, k_lo, default_prime(lx), SEEDS, nonce,
                            g=idx.astype(U64))
    assert np.array_equal(y0[idx], o0) and np.array_equal(y1[idx], o1)


def test_resnet18_ragged_batch_73859072(B, oracle_pool):
    """All 17 ReLU tensors of a ResNet-18 pass (batch 32) in one persistent
    launch replayed from a HIP graph, as bench.py runs it: property on every
    element, the oracle on every element of the largest tensor (32 x 64 x
    112^2) and on samples of the others."""
    from paper_2309_04909_amd import batch as BT
    prm = B.Params(64, 7, 11)
    data = W.resnet18_relu(seed=4, batch=32)
    segs = []
    for i, (_, (x0, x1)) in enumerate(data):
        d0, d1 = dev(x0), dev(x1)
        segs.append(BT.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=B.BC_OP_RELU, nonce=100 + i))
    assert sum(s.x0.numel() for s in segs) == 73859072
    rb = BT.RaggedBatch(prm, B.Seeds(*SEEDS), segs)
    graph = rb.capture()
    graph.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    for i, ((x, (x0, x1)), s) in enumerate(zip(data, segs)):
        y0, y1 = host(s.y0), host(s.y1)
        check_relu_property(recon(y0, y1, 64), x, signed(x, 64), 11)
        if i == 0:
            o0, o1 = protocol_all(oracle_pool, "relu", x0, x1, 64, 7, 11, 251, SEEDS, 100 + i)
            assert np.array_equal(y0, o0) and np.array_equal(y1, o1), "segment 0, every element"
            continue
        idx = sample_indices(x.size, rng, k=300)
        o0, o1, _, _ = OPR.relu(x0[idx], x1[idx], 64, 7, 11, 251, SEEDS, 100 + i, g=idx.astype(U64))
        assert np.array_equal(y0[idx], o0) and np.array_equal(y1[idx], o1), f"segment {i}"


@pytest.mark.parametrize("lx,k_lo", [(18, 13), (7, 11)])
def test_rss_keybit_2p24(B, lx, k_lo):
    """Replicated-sharing DReLU / ReLU on the 2^24 key-bit values, shared as
    bench.py shares them: the DReLU property on every element, the ReLU
    identity x DReLU(x) on every element, the oracle on samples."""
    x, (x0, x1), _, _ = W.keybit_drelu(seed=2, n=1 << 24)
    n = x.size
    a = np.random.default_rng(31).integers(0, 1 << 63, size=n, dtype=np.uint64) * U64(2)
    xs = (x0 - a, a, x1)
    d = tuple(dev(v) for v in xs)
    seeds5 = SEEDS + (0x5EED012, 0x5EED2)
    prm, sd = B.Params(64, lx, k_lo), B.RssSeeds(*seeds5, 41)
    yd = [host(t) for t in B.rss_drelu(d, prm, sd)]
    yr = [host(t) for t in B.rss_relu(d, prm, sd)]
    del d
    xi = signed(x, 64)
    dr = yd[0] + yd[1] + yd[2]
    if lx == 18:
        check_drelu_property(dr, xi, k_lo)
    else:
        # |x| < 2^30 exceeds this window's guard domain: only the bit property is fixed
        assert np.all((dr == 0) | (dr == 1))
    assert np.array_equal(yr[0] + yr[1] + yr[2], x * dr)
    idx = sample_indices(n, np.random.default_rng(9), k=1500)
    e, _, _ = OPR.rss_relu(*(v[idx] for v in xs), 64, lx, k_lo, default_prime(lx), seeds5, 41, g=idx.astype(U64))
    for j in range(3):
        assert np.array_equal(yr[j][idx], e[j])


def test_layer_chain_73859072(B, oracle_pool):
    """The bench's layer chain: all 17 ResNet-18 tensors as products (f = 26)
    in Z_2^64, truncated by 13 and ReLU'd in Z_2^51 by one batch launch with
    per-segment truncation, replayed from a HIP graph: equal to the fused
    single calls on every element, the oracle (Alg. 5 then Alg. 8) on every
    element of the largest tensor and on samples of the others."""
    from paper_2309_04909_amd import batch as BT
    prm = B.Params(51, 7, 11)
    data = W.resnet18_relu(seed=4, batch=32, f=26)
    segs = []
    for i, (_, (x0, x1)) in enumerate(data):
        d0, d1 = dev(x0), dev(x1)
        segs.append(BT.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=B.BC_OP_RELU, nonce=200 + i,
                               k_in=13))
    rb = BT.RaggedBatch(prm, B.Seeds(*SEEDS), segs)
    graph = rb.capture()
    graph.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(10)
    for i, ((_, (x0, x1)), s) in enumerate(zip(data, segs)):
        f0, f1 = B.trunc_relu(s.x0, s.x1, 64, 13, prm, B.Seeds(*SEEDS, s.nonce))
        assert torch.equal(f0.view(torch.int64), s.y0.view(torch.int64)), f"segment {i}"
        assert torch.equal(f1.view(torch.int64), s.y1.view(torch.int64)), f"segment {i}"
        if i == 0:
            o0, o1 = protocol_all(oracle_pool, "relu", x0, x1, 51, 7, 11, 251, SEEDS, 200 + i, k_in=13)
            assert np.array_equal(host(s.y0), o0) and np.array_equal(host(s.y1), o1), "segment 0, every element"
            continue
        idx = sample_indices(x0.size, rng, k=200)
        t0, t1 = OPR.trunc_det(x0[idx], x1[idx], 64, 13, 0)
        o0, o1, _, _ = OPR.relu(t0, t1, 51, 7, 11, 251, SEEDS, 200 + i, g=idx.astype(U64))
        assert np.array_equal(host(s.y0)[idx], o0) and np.array_equal(host(s.y1)[idx], o1), f"segment {i}"


@pytest.mark.parametrize("op", ["drelu", "relu"])
def test_call_above_one_launch(B, op):
    """A call of 2^28 + 5 elements runs as two launches (one launch indexes
    elements and byte offsets in 32 bits): outputs around the boundary and on
    random samples equal the oracle's (Alg. 7 / Alg. 8), and the elements past
    the boundary equal a call on them alone with their element offset."""
    lx, k_lo, half = 18, 13, 1 << 28
    n = half + 5
    prm = B.Params(64, lx, k_lo)
    nonce = 0xB16 + (op == "relu")
    sd = B.Seeds(*SEEDS, nonce)
    fn = B.relu if op == "relu" else B.drelu
    gen = torch.Generator(device="cuda").manual_seed(17)
    x0 = torch.randint(-(1 << 62), 1 << 62, (n,), device="cuda", dtype=torch.int64, generator=gen)
    x1 = torch.randint(-(1 << 62), 1 << 62, (n,), device="cuda", dtype=torch.int64, generator=gen)
    y0, y1 = (y.view(torch.int64) for y in fn(x0, x1, prm, sd))
    rng = np.random.default_rng(23)
    idx = np.unique(np.concatenate([np.arange(half - 3, n), np.arange(4), rng.integers(0, n, size=300)]))
    it = torch.from_numpy(idx.astype(np.int64)).cuda()
    xs0, xs1 = host(x0[it]), host(x1[it])
    ofn = OPR.relu if op == "relu" else OPR.drelu
    e0, e1, _, _ = ofn(xs0, xs1, 64, lx, k_lo, default_prime(lx), SEEDS, nonce, g=idx.astype(U64))
    assert np.array_equal(host(y0[it]), e0) and np.array_equal(host(y1[it]), e1)
    t0, t1 = fn(x0[half:], x1[half:], prm, sd, elem_base=half)
    assert torch.equal(t0.view(torch.int64), y0[half:])
    assert torch.equal(t1.view(torch.int64), y1[half:])
    del x0, x1, y0, y1
    torch.cuda.empty_cache()
