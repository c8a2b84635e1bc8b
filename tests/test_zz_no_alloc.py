"""The allocation-free ragged batch (bc_batch_run_static) against bc_batch_run.

Two calls in a row through the C ABI, the second on a smaller batch: each
must give, on every element of every segment, exactly the outputs of
bc_batch_run on the same plan (which the batch tests check against single
calls and the oracle), plus oracle samples here.  The first plan spans
several upload launches; the second overwrites only the front of the area,
so a stale tail of the first plan must not leak into it."""

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


def _batch(B, bt, rng, ell, lx, k_lo, sizes, k_in=0):
    """Segments of the given sizes (DReLU and ReLU alternating, every third
    truncating its inputs by k_in first), their inputs and a RaggedBatch."""
    segs, inputs = [], []
    base = 0
    for i, n in enumerate(sizes):
        kin = k_in if i % 3 == 2 else 0
        bound = 1 << (k_lo + lx - 1 + kin)
        x = np.array([v % (1 << (ell + kin)) for v in rng.integers(-bound + 1, bound, size=n).tolist()],
                     dtype=np.uint64 if ell > 32 else np.uint32)
        x0, x1 = W.share(x.astype(np.uint64), ell + kin, rng)
        dt = np.uint64 if ell > 32 else np.uint32
        d0, d1 = dev(x0.astype(dt)), dev(x1.astype(dt))
        op = B.BC_OP_RELU if i % 2 else B.BC_OP_DRELU
        segs.append(bt.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=op, nonce=31 + 5 * i,
                               elem_base=base, k_in=kin))
        inputs.append((x0, x1, kin))
        base += n + 7
    return segs, inputs


def _run_both(B, bt, prm, seeds, segs, inputs, lx, k_lo, ell):
    batch = bt.RaggedBatch(prm, B.Seeds(*seeds), segs)
    batch.run()                                     # bc_batch_run: device plan owned by the batch
    want = [(s.y0.clone(), s.y1.clone()) for s in segs]
    for s in segs:                                  # poison the outputs before the static run
        s.y0.fill_(-1)
        s.y1.fill_(-1)
    batch.run_static()                              # bc_batch_run_static: the fixed device area
    torch.cuda.synchronize()
    p = default_prime(lx)
    for s, (w0, w1), (x0, x1, kin) in zip(segs, want, inputs):
        assert torch.equal(s.y0, w0) and torch.equal(s.y1, w1), (s.x0.numel(), s.op, s.k_in)
        k = min(64, x0.size)
        if k:
            a0, a1 = x0[:k].astype(np.uint64), x1[:k].astype(np.uint64)
            if kin:
                a0, a1 = OPR.trunc_det(a0, a1, ell + kin, kin, 0)
            ofn = OPR.relu if s.op == B.BC_OP_RELU else OPR.drelu
            e0, e1, _, _ = ofn(a0, a1, ell, lx, k_lo, p, seeds, s.nonce, elem_base=s.elem_base)
            assert np.array_equal(host(s.y0)[:k].astype(np.uint64), e0)
            assert np.array_equal(host(s.y1)[:k].astype(np.uint64), e1)


def test_static_plan_two_calls_second_smaller(M):
    B, bt = M
    rng = np.random.default_rng(909)
    seeds = (71, 72, 73)
    # first call: 300 segments (a 21,672-byte plan: eight upload launches) in
    # Z_2^51, every third truncating shares of Z_2^64 by 13 bits first
    sizes = [int(v) for v in rng.integers(0, 3000, size=300)]
    sizes[:4] = [0, 1, 1023, 20000]
    segs, inputs = _batch(B, bt, rng, 51, 7, 11, sizes, k_in=13)
    _run_both(B, bt, B.Params(51, 7, 11), seeds, segs, inputs, 7, 11, 51)
    # second call: 5 smaller segments, another setting (l = 32, 32-bit storage)
    segs, inputs = _batch(B, bt, rng, 32, 8, 8, [1, 700, 0, 257, 64], k_in=0)
    _run_both(B, bt, B.Params(32, 8, 8), seeds, segs, inputs, 8, 8, 32)


def test_static_plan_largest(M):
    B, bt = M
    rng = np.random.default_rng(910)
    n_max = int(B.BC_STATIC_MAX_SEGMENTS)
    sizes = [int(v) for v in rng.integers(0, 40, size=n_max)]
    segs, inputs = _batch(B, bt, rng, 64, 18, 13, sizes)
    _run_both(B, bt, B.Params(64, 18, 13), (1, 2, 3), segs, inputs, 18, 13, 64)
