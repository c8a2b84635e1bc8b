"""Ragged batches on the GPU: one persistent launch gives, for every segment,
exactly the result of a single call on it (and of the oracle), under any tile
size or grid, and a captured graph replays it correctly."""

import numpy as np
import pytest

from oracle import protocols as OPR
from oracle.params import default_prime
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import batch, bicop
    return bicop, batch


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


SIZES = [0, 1, 255, 256, 1023, 1024, 1025, 5000, 77777, 3]


def _segments(B, bt, rng, ell, lx, k_lo, sizes, ops=None):
    segs, inputs = [], []
    base = 0
    for i, n in enumerate(sizes):
        bound = 1 << (k_lo + lx - 1)
        x = np.array([v % (1 << ell) for v in rng.integers(-bound + 1, bound, size=n).tolist()], dtype=np.uint64)
        x0, x1 = W.share(x, ell, rng)
        op = (ops[i] if ops else (B.BC_OP_RELU if i % 2 else B.BC_OP_DRELU))
        d0, d1 = dev(x0), dev(x1)
        segs.append(bt.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=op, nonce=1000 + 7 * i,
                               elem_base=base))
        inputs.append((x0, x1))
        base += n + 13
    return segs, inputs


@pytest.mark.parametrize("ell,lx,k_lo", [(64, 7, 11), (64, 18, 13), (32, 8, 8), (64, 32, 0)])
def test_batch_equals_single_calls_and_oracle(M, ell, lx, k_lo):
    B, bt = M
    rng = np.random.default_rng(ell + lx)
    prm, seeds = B.Params(ell, lx, k_lo), (5, 6, 7)
    segs, inputs = _segments(B, bt, rng, ell, lx, k_lo, SIZES)
    batch = bt.RaggedBatch(prm, B.Seeds(*seeds), segs)
    batch.run()
    p = default_prime(lx)
    for s, (x0, x1) in zip(segs, inputs):
        fn = B.relu if s.op == B.BC_OP_RELU else B.drelu
        z0, z1 = fn(s.x0, s.x1, prm, B.Seeds(*seeds, s.nonce), elem_base=s.elem_base)
        assert same(z0, s.y0) and same(z1, s.y1), (s.x0.numel(), s.op)
        k = min(400, x0.size)
        if k:
            ofn = OPR.relu if s.op == B.BC_OP_RELU else OPR.drelu
            e0, e1, _, _ = ofn(x0[:k].astype(np.uint64), x1[:k].astype(np.uint64), ell, lx, k_lo, p, seeds, s.nonce,
                               elem_base=s.elem_base)
            assert np.array_equal(host(s.y0)[:k].astype(np.uint64), e0)
            assert np.array_equal(host(s.y1)[:k].astype(np.uint64), e1)


def test_batch_schedule_invariance(M):
    B, bt = M
    rng = np.random.default_rng(3)
    prm = B.Params(64, 7, 11)
    segs, _ = _segments(B, bt, rng, 64, 7, 11, [3000, 10, 70000, 4096])
    ref = None
    for tile, grid in [(0, 0), (256, 1), (512, 3), (4096, 0), (100, 7)]:
        for s in segs:
            s.y0.zero_()
            s.y1.zero_()
        bt.RaggedBatch(prm, B.Seeds(1, 2, 3), segs, tile_elems=tile, grid=grid).run()
        out = [(s.y0.clone(), s.y1.clone()) for s in segs]
        if ref is None:
            ref = out
        else:
            for (a0, a1), (b0, b1) in zip(ref, out):
                assert same(a0, b0) and same(a1, b1), (tile, grid)


def test_batch_graph_replays(M):
    """Each replay of the captured launch reproduces the eager result, with eager
    work (clearing the outputs, other kernels) between replays."""
    B, bt = M
    rng = np.random.default_rng(4)
    prm = B.Params(64, 7, 11)
    segs, _ = _segments(B, bt, rng, 64, 7, 11, [20000, 513, 0, 40000])
    batch = bt.RaggedBatch(prm, B.Seeds(9, 8, 7), segs)
    batch.run()
    torch.cuda.synchronize()
    eager = [(s.y0.clone(), s.y1.clone()) for s in segs]
    g = batch.capture()
    for rep in range(4):
        for s in segs:
            s.y0.zero_()
            s.y1.zero_()
        junk = torch.randn(4096, device="cuda").sum()          # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for (a0, a1), s in zip(eager, segs):
            assert same(a0, s.y0) and same(a1, s.y1), rep


def test_graph_keeps_its_plan_alive(M):
    """A graph captured from a batch that the caller does not keep still
    replays correctly after the allocator has handed out (and overwritten)
    fresh memory: the graph holds the batch, and with it the device plan."""
    import gc
    B, bt = M
    rng = np.random.default_rng(12)
    prm = B.Params(64, 7, 11)
    segs, _ = _segments(B, bt, rng, 64, 7, 11, [30000, 777, 5000])
    g = bt.RaggedBatch(prm, B.Seeds(3, 4, 5), segs).capture()
    gc.collect()
    churn = [torch.full((n,), -1, dtype=torch.int64, device="cuda") for n in (64, 512, 4096, 1 << 16)]
    for s in segs:
        s.y0.zero_()
        s.y1.zero_()
    g.replay()
    torch.cuda.synchronize()
    for s in segs:
        fn = B.relu if s.op == B.BC_OP_RELU else B.drelu
        z0, z1 = fn(s.x0, s.x1, prm, B.Seeds(3, 4, 5, s.nonce), elem_base=s.elem_base)
        assert same(z0, s.y0) and same(z1, s.y1)
    del churn


@pytest.mark.parametrize("ell_in,k_in,lx,k_lo", [(64, 13, 11, 13), (32, 8, 7, 10), (64, 20, 7, 11)])
def test_batch_with_input_truncation(M, ell_in, k_in, lx, k_lo):
    """A layer chain in one launch: segments whose inputs are products in
    Z_2^ell_in, truncated by k_in bits first (Alg. 5), mixed with segments
    already in the ring.  Each equals bc_trunc_drelu / bc_trunc_relu (or the
    plain call) on its own, and the oracle on samples."""
    B, bt = M
    ell = ell_in - k_in
    rng = np.random.default_rng(ell_in + k_in)
    prm, seeds = B.Params(ell, lx, k_lo), (15, 16, 17)
    sizes = [5000, 0, 1, 77777, 1025, 4096]
    segs, inputs, base = [], [], 0
    for i, n in enumerate(sizes):
        kin = k_in if i % 3 != 1 else 0
        ring = ell + kin
        bound = 1 << (k_lo + lx - 2 + kin)
        x = np.array([v % (1 << ring) for v in rng.integers(-bound + 1, bound, size=n).tolist()], dtype=np.uint64)
        x0, x1 = W.share(x, ring, rng)
        op = B.BC_OP_RELU if i % 2 else B.BC_OP_DRELU
        d0, d1 = dev(x0), dev(x1)
        segs.append(bt.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=op, nonce=300 + i,
                               elem_base=base, k_in=kin))
        inputs.append((x0, x1))
        base += n + 5
    bt.RaggedBatch(prm, B.Seeds(*seeds), segs).run()
    p = default_prime(lx)
    for s, (x0, x1) in zip(segs, inputs):
        sd = B.Seeds(*seeds, s.nonce)
        if s.k_in:
            fn = B.trunc_relu if s.op == B.BC_OP_RELU else B.trunc_drelu
            z0, z1 = fn(s.x0, s.x1, ell + s.k_in, s.k_in, prm, sd, elem_base=s.elem_base)
        else:
            fn = B.relu if s.op == B.BC_OP_RELU else B.drelu
            z0, z1 = fn(s.x0, s.x1, prm, sd, elem_base=s.elem_base)
        assert same(z0, s.y0) and same(z1, s.y1), (s.x0.numel(), s.k_in)
        k = min(300, x0.size)
        if k:
            t0, t1 = OPR.trunc_det(x0[:k].astype(np.uint64), x1[:k].astype(np.uint64), ell + s.k_in, s.k_in, 0)
            ofn = OPR.relu if s.op == B.BC_OP_RELU else OPR.drelu
            e0, e1, _, _ = ofn(t0, t1, ell, lx, k_lo, p, seeds, s.nonce, elem_base=s.elem_base)
            assert np.array_equal(host(s.y0)[:k].astype(np.uint64), e0)
            assert np.array_equal(host(s.y1)[:k].astype(np.uint64), e1)


@pytest.mark.parametrize("ell_in,k_in,lx,k_lo", [(64, 13, 7, 11), (64, 13, 18, 13), (32, 8, 7, 10), (64, 0, 18, 13)])
def test_batch_with_records(M, ell_in, k_in, lx, k_lo):
    """A layer chain on precomputed randomness: segments whose records were
    expanded offline (bc_rand_expand with their own nonce and elem_base)
    mixed with segments drawing from the seeds, with and without input
    truncation.  A record segment equals bc_trunc_relu / bc_trunc_drelu (or
    the plain call) with the same seeds, nonce and elem_base.  Oracle on
    samples."""
    B, bt = M
    ell = ell_in - k_in
    rng = np.random.default_rng(7 * ell_in + k_in + lx)
    prm, seeds = B.Params(ell, lx, k_lo), (25, 26, 27)
    sizes = [4097, 0, 1, 30000, 1025, 256, 9999]
    segs, inputs, base = [], [], 0
    for i, n in enumerate(sizes):
        kin = k_in if i % 3 != 1 else 0
        ring = ell + kin
        bound = 1 << (k_lo + lx - 2 + kin)
        x = np.array([v % (1 << ring) for v in rng.integers(-bound + 1, bound, size=n).tolist()], dtype=np.uint64)
        x0, x1 = W.share(x, ring, rng)
        op = B.BC_OP_RELU if i % 2 else B.BC_OP_DRELU
        d0, d1 = dev(x0), dev(x1)
        nonce, eb = 500 + i, base
        rec = None
        if i % 2 == 0 or i == 3:              # records on most segments; the rest draw from the seeds
            rec = B.rand_expand(op, prm, B.Seeds(*seeds, nonce), n, elem_base=eb)
        seg = bt.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=op, nonce=nonce, elem_base=eb,
                         k_in=kin, rand=rec)
        segs.append(seg)
        inputs.append((x0, x1, nonce, eb))
        base += n + 3
    bt.RaggedBatch(prm, B.Seeds(*seeds), segs).run()
    torch.cuda.synchronize()
    p = default_prime(lx)
    for s, (x0, x1, nonce, eb) in zip(segs, inputs):
        sd = B.Seeds(*seeds, nonce)
        if s.k_in:
            fn = B.trunc_relu if s.op == B.BC_OP_RELU else B.trunc_drelu
            z0, z1 = fn(s.x0, s.x1, ell + s.k_in, s.k_in, prm, sd, elem_base=eb)
        else:
            fn = B.relu if s.op == B.BC_OP_RELU else B.drelu
            z0, z1 = fn(s.x0, s.x1, prm, sd, elem_base=eb)
        assert same(z0, s.y0) and same(z1, s.y1), (s.x0.numel(), s.k_in, s.rand is not None)
        k = min(200, x0.size)
        if k:
            t0, t1 = x0[:k].astype(np.uint64), x1[:k].astype(np.uint64)
            if s.k_in:
                t0, t1 = OPR.trunc_det(t0, t1, ell + s.k_in, s.k_in, 0)
            ofn = OPR.relu if s.op == B.BC_OP_RELU else OPR.drelu
            e0, e1, _, _ = ofn(t0, t1, ell, lx, k_lo, p, seeds, nonce, elem_base=eb)
            assert np.array_equal(host(s.y0)[:k].astype(np.uint64), e0)
            assert np.array_equal(host(s.y1)[:k].astype(np.uint64), e1)


def test_batch_record_graph_replays(M):
    """A captured batch with record segments replays the eager result."""
    B, bt = M
    rng = np.random.default_rng(14)
    prm = B.Params(64, 7, 11)
    segs, _ = _segments(B, bt, rng, 64, 7, 11, [20000, 513, 40000])
    for i, s in enumerate(segs):
        if i != 1:
            s.rand = B.rand_expand(s.op, prm, B.Seeds(9, 8, 7, s.nonce), s.x0.numel(), elem_base=s.elem_base)
    batch = bt.RaggedBatch(prm, B.Seeds(9, 8, 7), segs)
    batch.run()
    torch.cuda.synchronize()
    eager = [(s.y0.clone(), s.y1.clone()) for s in segs]
    for s in segs:
        fn = B.relu if s.op == B.BC_OP_RELU else B.drelu
        z0, z1 = fn(s.x0, s.x1, prm, B.Seeds(9, 8, 7, s.nonce), elem_base=s.elem_base)
        assert same(z0, s.y0) and same(z1, s.y1)
    g = batch.capture()
    for rep in range(3):
        for s in segs:
            s.y0.zero_()
            s.y1.zero_()
        g.replay()
        torch.cuda.synchronize()
        for (a0, a1), s in zip(eager, segs):
            assert same(a0, s.y0) and same(a1, s.y1), rep
