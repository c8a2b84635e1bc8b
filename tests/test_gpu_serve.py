"""Serving: every job's result is identical alone and in the mix (tolerance 0),
and a sample of jobs matches the oracle."""

import numpy as np
import pytest

from oracle import protocols as OPR
from oracle.params import default_prime
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def test_results_identical_alone_and_in_the_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop as B
    from paper_2309_04909_amd import serve as S
    pool_n = 1 << 18
    settings = {64: (64, 18, 13), 32: (32, 8, 8)}
    host_pools, pools = {}, {}
    for ell in (64, 32):
        _, (x0, x1) = W.serving_values(50 + ell, pool_n, ell)
        host_pools[ell] = (x0, x1)
        pools[ell] = (dev(x0), dev(x1))
    params = {ell: B.Params(*settings[ell]) for ell in settings}
    seeds = (31, 41, 59)
    rng = np.random.default_rng(0)
    arr = W.serving_arrivals(3, 20000.0, 60, min_log2=4, max_log2=16)
    jobs = []
    for i, (t, n, op, ell) in enumerate(arr):
        jobs.append(S.Job(i, t, n, 0 if op == "drelu" else 1, ell, int(rng.integers(0, pool_n - n + 1)), 7000 + i))
    # a tight budget and few slots force many small launches that overlap on 3 streams
    srv = S.Server(pools, params, B.Seeds(*seeds), hbm_budget=1 << 22, max_slots=5, nstreams=3, keep_outputs=True)
    srv.warmup()                                            # kernels loaded, outputs reserved, plan buffers pinned
    assert len(srv._pinned) == 2 * 3
    done = srv.run(jobs)
    assert len(srv._pinned) >= 2 * 3                        # every launch's plan buffer came back
    assert len(done) == len(jobs) and all(j.done is not None and j.done >= j.arrival - 1e-3 for j in done)
    for j in done:
        x0, x1 = pools[j.ell]
        fn = B.relu if j.op == B.BC_OP_RELU else B.drelu
        a0, a1 = fn(x0[j.offset:j.offset + j.n], x1[j.offset:j.offset + j.n], params[j.ell], B.Seeds(*seeds, j.nonce))
        assert same(a0, j.y0) and same(a1, j.y1), j.jid
    for j in done[:6]:
        ell, lx, k_lo = settings[j.ell]
        h0, h1 = host_pools[j.ell]
        k = min(j.n, 300)
        ofn = OPR.relu if j.op == B.BC_OP_RELU else OPR.drelu
        e0, e1, _, _ = ofn(h0[j.offset:j.offset + k].astype(np.uint64), h1[j.offset:j.offset + k].astype(np.uint64),
                           ell, lx, k_lo, default_prime(lx), seeds, j.nonce)
        assert np.array_equal(host(j.y0)[:k].astype(np.uint64), e0)
        assert np.array_equal(host(j.y1)[:k].astype(np.uint64), e1)


def test_arena_outputs_in_the_mix():
    """Without keep_outputs the launches write into the output arena, whose
    ranges are reused as launches retire (a budget this small forces many
    reuses); each job's result, copied out in the on_done callback before its
    range is released, equals the single call on that job."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop as B
    from paper_2309_04909_amd import serve as S
    pool_n = 1 << 18
    settings = {64: (64, 18, 13), 32: (32, 8, 8)}
    pools = {}
    for ell in (64, 32):
        _, (x0, x1) = W.serving_values(90 + ell, pool_n, ell)
        pools[ell] = (dev(x0), dev(x1))
    params = {ell: B.Params(*settings[ell]) for ell in settings}
    seeds = (71, 72, 73)
    rng = np.random.default_rng(5)
    arr = W.serving_arrivals(6, 20000.0, 80, min_log2=4, max_log2=16)
    jobs = [S.Job(i, t, n, 0 if op == "drelu" else 1, ell, int(rng.integers(0, pool_n - n + 1)), 5000 + i)
            for i, (t, n, op, ell) in enumerate(arr)]
    got = {}

    def collect(j, y0, y1):
        got[j.jid] = (y0.cpu(), y1.cpu())                  # a synchronous copy: done before the range is reused

    srv = S.Server(pools, params, B.Seeds(*seeds), hbm_budget=1 << 22, max_slots=6, nstreams=3, on_done=collect)
    srv.warmup()
    assert srv._arena is not None and srv._arena.numel() == (1 << 22) // 2
    done = srv.run(jobs)
    assert len(done) == len(jobs) and len(got) == len(jobs) and not srv._arena_used
    assert all(j.y0 is None and j.out is None for j in done)
    for j in done:
        x0, x1 = pools[j.ell]
        fn = B.relu if j.op == B.BC_OP_RELU else B.drelu
        a0, a1 = fn(x0[j.offset:j.offset + j.n], x1[j.offset:j.offset + j.n], params[j.ell], B.Seeds(*seeds, j.nonce))
        assert same(a0.cpu(), got[j.jid][0]) and same(a1.cpu(), got[j.jid][1]), j.jid


def test_precomputed_randomness_in_the_mix():
    """Jobs whose randomness was expanded offline (resident records, about half
    of them by the budget) run the online kernel; every result still equals
    the single fused call on that job."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop as B
    from paper_2309_04909_amd import serve as S
    pool_n = 1 << 18
    settings = {64: (64, 18, 13), 32: (32, 8, 8)}
    pools = {}
    for ell in (64, 32):
        _, (x0, x1) = W.serving_values(60 + ell, pool_n, ell)
        pools[ell] = (dev(x0), dev(x1))
    params = {ell: B.Params(*settings[ell]) for ell in settings}
    seeds = (27, 18, 28)
    rng = np.random.default_rng(1)
    arr = W.serving_arrivals(4, 20000.0, 60, min_log2=4, max_log2=16)
    jobs = [S.Job(i, t, n, 0 if op == "drelu" else 1, ell, int(rng.integers(0, pool_n - n + 1)), 9000 + i)
            for i, (t, n, op, ell) in enumerate(arr)]
    total = sum(B.rand_bytes(j.op, params[j.ell], j.n) for j in jobs)
    srv = S.Server(pools, params, B.Seeds(*seeds), hbm_budget=1 << 22, max_slots=5, nstreams=3, keep_outputs=True,
                   rand_budget=int(total * 0.4))
    with_rec, used, _ = srv.prepare(jobs)
    assert 0 < with_rec < len(jobs) and used <= int(total * 0.4)
    done = srv.run(jobs)
    assert len(done) == len(jobs) and all(j.rand is None for j in done)
    for j in done:
        x0, x1 = pools[j.ell]
        fn = B.relu if j.op == B.BC_OP_RELU else B.drelu
        a0, a1 = fn(x0[j.offset:j.offset + j.n], x1[j.offset:j.offset + j.n], params[j.ell], B.Seeds(*seeds, j.nonce))
        assert same(a0, j.y0) and same(a1, j.y1), j.jid


def test_layer_chain_jobs_with_records_in_the_mix():
    """Truncate-then-DReLU/ReLU jobs of a layer chain (products in Z_2^64,
    truncated by 13 bits into Z_2^51 inside the launch) served beside plain
    l = 64 and l = 32 jobs, about 40% of all jobs on resident records: each
    result equals the single fused call on that job (bc_trunc_relu /
    bc_trunc_drelu or bc_relu / bc_drelu), and chain jobs match the oracle on
    samples."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop as B
    from paper_2309_04909_amd import serve as S
    pool_n = 1 << 18
    settings = {64: (64, 18, 13), 32: (32, 8, 8), 51: (51, 7, 11)}
    host_pools, pools = {}, {}
    for ell in (64, 32):
        _, (x0, x1) = W.serving_values(70 + ell, pool_n, ell)
        host_pools[ell] = (x0, x1)
        pools[ell] = (dev(x0), dev(x1))
    _, (c0, c1) = W.chain_values(81, pool_n)             # f = 26 products, truncated by 13 into Z_2^51
    host_pools[51] = (c0, c1)
    pools[51] = (dev(c0), dev(c1))
    params = {ell: B.Params(*settings[ell]) for ell in settings}
    seeds = (11, 12, 13)
    rng = np.random.default_rng(2)
    arr = W.serving_arrivals(5, 20000.0, 72, min_log2=4, max_log2=16)
    jobs = []
    for i, (t, n, op, ell) in enumerate(arr):
        key, k_in = (51, 13) if i % 3 == 0 else (ell, 0)
        jobs.append(S.Job(i, t, n, 0 if op == "drelu" else 1, key, int(rng.integers(0, pool_n - n + 1)), 4000 + i,
                          k_in=k_in))
    total = sum(B.rand_bytes(j.op, params[j.ell], j.n) for j in jobs)
    srv = S.Server(pools, params, B.Seeds(*seeds), hbm_budget=1 << 22, max_slots=6, nstreams=3, keep_outputs=True,
                   rand_budget=int(total * 0.4))
    with_rec, _, _ = srv.prepare(jobs)
    assert 0 < with_rec < len(jobs)
    chain_rec = sum(1 for j in jobs if j.k_in and j.rand is not None)
    assert chain_rec > 0
    done = srv.run(jobs)
    assert len(done) == len(jobs) and all(j.rand is None for j in done)
    for j in done:
        x0, x1 = pools[j.ell]
        a, b = x0[j.offset:j.offset + j.n], x1[j.offset:j.offset + j.n]
        sd = B.Seeds(*seeds, j.nonce)
        relu = j.op == B.BC_OP_RELU
        if j.k_in:
            fn = B.trunc_relu if relu else B.trunc_drelu
            z0, z1 = fn(a, b, j.ell + j.k_in, j.k_in, params[j.ell], sd)
        else:
            z0, z1 = (B.relu if relu else B.drelu)(a, b, params[j.ell], sd)
        assert same(z0, j.y0) and same(z1, j.y1), (j.jid, j.ell, j.k_in)
    for j in [j for j in done if j.k_in][:4]:
        ell, lx, k_lo = settings[j.ell]
        h0, h1 = host_pools[j.ell]
        k = min(j.n, 200)
        t0, t1 = OPR.trunc_det(h0[j.offset:j.offset + k].astype(np.uint64), h1[j.offset:j.offset + k].astype(np.uint64),
                               64, 13, 0)
        ofn = OPR.relu if j.op == B.BC_OP_RELU else OPR.drelu
        e0, e1, _, _ = ofn(t0, t1, ell, lx, k_lo, default_prime(lx), seeds, j.nonce)
        assert np.array_equal(host(j.y0)[:k].astype(np.uint64), e0)
        assert np.array_equal(host(j.y1)[:k].astype(np.uint64), e1)
