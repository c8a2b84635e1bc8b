"""Run the CPU oracle over every element of a full-size workload, in chunks.

The oracle is vectorised over elements and draws each element's randomness
from its global index, so a workload splits into independent chunks.  With a
process pool (forked by conftest.py before the test session touches the GPU)
the chunks run in parallel; without one they run here, one after another.
This module only cuts arrays into chunks and joins the results: every value
comes from ``oracle``."""

import numpy as np

CHUNK = 1 << 18


def _worker(tasks, results):
    while True:
        item = tasks.get()
        if item is None:
            return
        i, fn, args = item
        try:
            results.put((i, True, fn(args)))
        except Exception as e:          # reported to the caller, which fails the test
            results.put((i, False, repr(e)))


class OraclePool:
    """A fixed set of forked worker processes.  Unlike multiprocessing.Pool it
    never forks a replacement: all workers exist from the start, so none is
    ever created from a process that has touched the GPU.  A worker that dies
    makes map() fail instead."""

    def __init__(self, workers):
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        self.tasks, self.results = ctx.Queue(), ctx.Queue()
        self.procs = [ctx.Process(target=_worker, args=(self.tasks, self.results), daemon=True)
                      for _ in range(workers)]
        for pr in self.procs:
            pr.start()

    def map(self, fn, jobs):
        import queue
        for i, j in enumerate(jobs):
            self.tasks.put((i, fn, j))
        out = [None] * len(jobs)
        for _ in jobs:
            while True:
                try:
                    i, ok, r = self.results.get(timeout=10)
                    break
                except queue.Empty:
                    dead = [pr.pid for pr in self.procs if not pr.is_alive()]
                    if dead:
                        raise RuntimeError(f"oracle workers died: {dead}")
            if not ok:
                raise RuntimeError(f"oracle chunk {i} failed: {r}")
            out[i] = r
        return out

    def close(self):
        for _ in self.procs:
            self.tasks.put(None)
        for pr in self.procs:
            pr.join(timeout=10)
            if pr.is_alive():
                pr.terminate()


def _chunk(args):
    op, x0, x1, ell, lx, k_lo, p, seeds, nonce, g, k_in = args
    from oracle import protocols as OPR
    if k_in:
        # Alg. 5 by k_in bits into Z_2^ell, then the protocol (a layer chain's step)
        x0, x1 = OPR.trunc_det(x0, x1, ell + k_in, k_in, 0)
    fn = OPR.relu if op == "relu" else OPR.drelu
    y0, y1, _, _ = fn(x0, x1, ell, lx, k_lo, p, seeds, nonce, g=g)
    return y0, y1


def protocol_all(pool, op, x0, x1, ell, lx, k_lo, p, seeds, nonce, elem_base=0, k_in=0, chunk=CHUNK):
    """The oracle's DReLU ("drelu") or ReLU ("relu") output shares of every
    element of (x0, x1), whose element i has global index elem_base + i."""
    x0 = np.asarray(x0, dtype=np.uint64)
    x1 = np.asarray(x1, dtype=np.uint64)
    n = x0.size
    jobs = []
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        g = np.arange(a, b, dtype=np.uint64) + np.uint64(elem_base)
        jobs.append((op, x0[a:b], x1[a:b], ell, lx, k_lo, p, seeds, nonce, g, k_in))
    res = pool.map(_chunk, jobs) if pool is not None else [_chunk(j) for j in jobs]
    if not res:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint64)
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])
