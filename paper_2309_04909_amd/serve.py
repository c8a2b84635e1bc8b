"""Continuous-batching request loop for DReLU/ReLU jobs.

Jobs (op, ring, n elements) arrive over time.  Their input shares live in a
device-resident pool (a job names a slice of it and carries its own nonce).
The loop:
  1. retires launches whose completion event has fired, freeing their slots
     and HBM;
  2. queues every job whose arrival time has passed;
  3. admits queued jobs in arrival order while the in-flight HBM (input and
     output shares of every admitted job) stays within the budget and slots
     are free;
  4. turns the newly admitted jobs into one ragged launch per ring
     (RaggedBatch, one persistent kernel each; a ring with a single job gets
     the plain call, which needs no plan) on the next of k streams, so work
     admitted while earlier launches run overlaps with them on the GPU.
Latency of a job = GPU completion time of its launch - its arrival time.
Each job's result is exactly what a single call on it would give (per-job
nonce, element indices 0..n-1), whichever launch it lands in.

A job may be one step of a layer chain: with k_in > 0 its inputs are shares
of Z_2^(ell + k_in) (a product at 2f fractional bits, say) that each party
first truncates by k_in bits (Alg. 5) inside the same launch; its result is
that of bc_trunc_drelu / bc_trunc_relu.

With a randomness budget, prepare() runs the offline phase before the
arrivals: it expands the seeds' draws of jobs (in arrival order, while they
fit the budget) into records kept resident in HBM.  Those jobs then run the
online kernel on their shares and record (inside the ragged launch of their
ring, or bc_drelu_pre / bc_relu_pre when alone), with the same results; a
record is released when its launch has completed.
"""

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field

import torch

from . import batch as BT
from . import bicop as B


@dataclass
class Job:
    jid: int
    arrival: float          # seconds after the start of the run
    n: int
    op: int                 # B.BC_OP_DRELU / B.BC_OP_RELU
    ell: int
    offset: int             # first element of its input slice in the pool of its ring
    nonce: int
    y0: torch.Tensor = None
    y1: torch.Tensor = None
    done: float = None      # completion time (s after the start)
    admitted: float = None
    rand: torch.Tensor = None   # resident randomness record (prepare), or None
    k_in: int = 0               # truncate the input shares by k_in bits first (a layer chain's step)
    out: tuple = None           # (y0, y1, first element) of its launch's output buffers while in flight


@dataclass
class Launch:
    event: torch.cuda.Event
    jobs: list
    batches: list = field(default_factory=list)
    records: list = field(default_factory=list)   # kept alive until the launch has completed
    outputs: list = field(default_factory=list)   # the launch's output buffers, one pair per ring
    pinned: list = field(default_factory=list)    # its (pinned, device) plan buffers, reused once it has completed
    arena: list = field(default_factory=list)     # start offsets of its output ranges in the arena
    bytes: int = 0


class Server:
    def __init__(self, pools, params, seeds: B.Seeds, hbm_budget: int, max_slots: int = 256, nstreams: int = 4,
                 keep_outputs: bool = False, rand_budget: int = 0, on_done=None, max_batch: int = 0):
        """pools[ell] = (x0, x1) device share pools; params[ell] = B.Params of that ring;
        rand_budget = HBM bytes for resident randomness records (0 = none).
        max_batch = jobs per launch (default max_slots / (4 nstreams), so
        that several launches are in flight and a retiring one frees slots for
        the next while the others still run; 8 to 32 jobs per launch measured
        alike, and 64 lost a quarter of the saturated throughput).
        With keep_outputs every job keeps its own output tensors (job.y0,
        job.y1); otherwise outputs live in an arena and are released when the
        job's launch has completed, after on_done(job, y0, y1) (if given) has
        returned: the callback must have finished reading them by then (copy
        to the host, or clone and synchronize)."""
        self.on_done = on_done
        self.rand_budget = rand_budget
        self.pools = pools
        self.params = params
        self.seeds = seeds
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.max_batch = max_batch if max_batch > 0 else max(1, max_slots // (4 * nstreams))
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.keep = keep_outputs
        self._events = []                            # completion events of retired launches, reused
        self._pinned = []                            # (pinned, device) plan buffers of retired launches, reused
        self._arena = None                           # output arena (half the budget), without keep_outputs
        self._arena_used = []                        # its ranges in flight: sorted (start, end) byte offsets

    def warmup(self):
        """One small call per ring, op and lane-group size, so that no job pays
        for loading a kernel's code object on its first launch; the output
        arena and the pinned plan buffers allocated up front, so that no launch
        waits for an allocation."""
        if not self.keep:
            self._make_arena(next(iter(self.pools.values()))[0].device)
        need = BT.RaggedBatch.plan_bytes(self.max_slots)
        dev = next(iter(self.pools.values()))[0].device
        while len(self._pinned) < 2 * len(self.streams):        # a plan per ring and stream
            self._pinned.append((torch.empty(need, dtype=torch.uint8, pin_memory=True),
                                 torch.empty(need, dtype=torch.uint8, device=dev)))
        for ell, (x0, x1) in self.pools.items():
            prm = self.params[ell]
            for fn in (B.drelu, B.relu):
                for n in (100, 12000, 70000):
                    m = min(n, x0.numel())
                    fn(x0[:m], x1[:m], prm, self.seeds)
            m = min(1000, x0.numel())
            ys = [torch.empty_like(x0[:m]) for _ in range(4)]
            segs = [BT.Segment(x0[:m], x1[:m], ys[0], ys[1], op=B.BC_OP_DRELU),
                    BT.Segment(x0[:m], x1[:m], ys[2], ys[3], op=B.BC_OP_RELU)]
            if self.rand_budget:
                for sg in segs:
                    sg.rand = B.rand_expand(sg.op, prm, self.seeds, m)
                B.drelu_pre(x0[:m], x1[:m], prm, segs[0].rand)
                B.relu_pre(x0[:m], x1[:m], prm, segs[1].rand)
            BT.RaggedBatch(prm, self.seeds, segs).run()
        torch.cuda.synchronize()

    def _seeds(self, nonce):
        return B.Seeds(self.seeds.seed01, self.seeds.seed02, self.seeds.seed12, nonce)

    def prepare(self, jobs):
        """Offline phase: records for jobs in arrival order while they fit the
        randomness budget.  Returns (jobs given a record, record bytes, seconds)."""
        t = time.perf_counter()
        used = count = 0
        for j in sorted(jobs, key=lambda j: j.arrival):
            nb = B.rand_bytes(j.op, self.params[j.ell], j.n)
            if used + nb > self.rand_budget:
                continue
            j.rand = B.rand_expand(j.op, self.params[j.ell], self._seeds(j.nonce), j.n)
            used += nb
            count += 1
        torch.cuda.synchronize()
        return count, used, time.perf_counter() - t

    def job_bytes(self, j: Job) -> int:
        return 4 * j.n * B.ring_width(j.ell)           # resident input shares + output shares

    def _check_slice(self, j: Job):
        x0 = self.pools[j.ell][0]
        if j.n < 1 or j.offset < 0 or j.offset + j.n > x0.numel():
            raise ValueError(f"job {j.jid}: elements [{j.offset}, {j.offset + j.n}) outside the pool of ring {j.ell}")

    def _launch(self, jobs, stream):
        """One launch for the admitted jobs: per ring, one pair of output
        buffers and one ragged batch built straight from raw segment records
        (pointers into the ring's pool and the output buffers), or the plain
        call for a ring with a single job."""
        ev = self._events.pop() if self._events else torch.cuda.Event(enable_timing=True)
        L = Launch(ev, jobs)
        m = (1 << 64) - 1
        with torch.cuda.stream(stream):
            by_ell = {}
            for j in jobs:
                L.bytes += self.job_bytes(j)
                by_ell.setdefault(j.ell, []).append(j)
            for ell, js in by_ell.items():
                x0, x1 = self.pools[ell]
                prm = self.params[ell]
                w = x0.element_size()
                total = sum(j.n for j in js)
                y0, y1 = self._outputs(total, x0, stream, L)
                L.outputs.append((y0, y1))
                if len(js) == 1 and not (js[0].rand is not None and js[0].k_in):
                    j = js[0]                            # one job: the plain call needs no plan
                    j.out = (y0, y1, 0)
                    self._single(j, prm, x0[j.offset:j.offset + j.n], x1[j.offset:j.offset + j.n], y0, y1, stream)
                    if j.rand is not None:
                        L.records.append(j.rand)
                        j.rand = None
                    continue
                recs = (B._Segment * len(js))()
                p0, p1, q0, q1 = x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr()
                off = 0
                for i, j in enumerate(js):
                    rp = rd = None
                    if j.rand is not None:               # released with the launch, once it has completed
                        rp, rd = j.rand.data_ptr(), ctypes.pointer(B.rand_desc(j.rand))
                        L.records.append(j.rand)
                        j.rand = None
                    recs[i] = B._Segment(p0 + w * j.offset, p1 + w * j.offset, q0 + w * off, q1 + w * off, j.n, 0,
                                         j.nonce & m, j.op, j.k_in, rp, rd)
                    j.out = (y0, y1, off)
                    off += j.n
                hp, dp = self._plan_buffer(len(js), x0.device)
                L.pinned.append((hp, dp))
                rb = BT.RaggedBatch.from_records(prm, self.seeds, recs, x0.device, total, host_plan=hp, dev_plan=dp)
                rb.run(stream)
                L.batches.append(rb)
            ev.record(stream)
        return L

    def _plan_buffer(self, nseg, device):
        """A (pinned, device) buffer pair for a plan of nseg segments: a
        retired launch's, or a new pair sized for max_slots segments.  Both
        allocations are slow (a device allocation can wait for the whole
        device), so warmup makes one pair per ring and stream up front."""
        need = BT.RaggedBatch.plan_bytes(nseg)
        for i, (h, _) in enumerate(self._pinned):
            if h.numel() >= need:
                return self._pinned.pop(i)
        size = max(need, BT.RaggedBatch.plan_bytes(self.max_slots))
        return (torch.empty(size, dtype=torch.uint8, pin_memory=True),
                torch.empty(size, dtype=torch.uint8, device=device))

    def _make_arena(self, device):
        if self._arena is None:
            self._arena = torch.empty(max(self.budget // 2, 256), dtype=torch.uint8, device=device)

    def _arena_alloc(self, nbytes):
        """First fit of nbytes (rounded to 256) among the ranges in flight, or None."""
        nbytes = (nbytes + 255) & ~255
        start = 0
        for i, (a, b) in enumerate(self._arena_used):
            if a - start >= nbytes:
                self._arena_used.insert(i, (start, start + nbytes))
                return start
            start = b
        if self._arena.numel() - start >= nbytes:
            self._arena_used.append((start, start + nbytes))
            return start
        return None

    def _arena_free(self, start):
        for i, (a, _) in enumerate(self._arena_used):
            if a == start:
                del self._arena_used[i]
                return

    def _outputs(self, total, like, stream, L):
        """A launch's output pair for one ring.  Without keep_outputs: a range
        of the output arena, free again once the launch has completed (the
        budget bounds the output bytes in flight by the arena's size; only
        fragmentation can make it fall back).  Otherwise, or on that
        fallback: new tensors of the launch's stream, which outlive it."""
        w = like.element_size()
        if not self.keep:
            self._make_arena(like.device)
            start = self._arena_alloc(2 * total * w)
            if start is not None:
                L.arena.append(start)
                a = self._arena
                return (a[start:start + total * w].view(like.dtype),
                        a[start + total * w:start + 2 * total * w].view(like.dtype))
        with torch.cuda.stream(stream):
            return (torch.empty(total, dtype=like.dtype, device=like.device),
                    torch.empty(total, dtype=like.dtype, device=like.device))

    def _single(self, j, prm, x0, x1, y0, y1, stream):
        out = (y0, y1)
        relu = j.op == B.BC_OP_RELU
        if j.rand is not None:                       # online kernel on the resident record
            fn = B.relu_pre if relu else B.drelu_pre
            fn(x0, x1, prm, j.rand, out=out, stream=stream)
        elif j.k_in:
            fn = B.trunc_relu if relu else B.trunc_drelu
            fn(x0, x1, prm.ell + j.k_in, j.k_in, prm, self._seeds(j.nonce), out=out, stream=stream)
        else:
            fn = B.relu if relu else B.drelu
            fn(x0, x1, prm, self._seeds(j.nonce), out=out, stream=stream)

    def run(self, jobs):
        """Serve `jobs` (arrival times relative to the start); returns them with
        completion times filled in."""
        for j in jobs:
            self._check_slice(j)
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting = deque()
        inflight = []
        used, slots, k = 0, 0, 0
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        t0 = time.perf_counter()
        finished = []
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            still = []
            for L in inflight:
                if L.event.query():
                    t_done = ref.elapsed_time(L.event) / 1e3
                    for j in L.jobs:
                        j.done = t_done
                        y0, y1, off = j.out
                        if self.keep:
                            j.y0, j.y1 = y0[off:off + j.n], y1[off:off + j.n]
                        if self.on_done is not None:
                            self.on_done(j, y0[off:off + j.n], y1[off:off + j.n])
                        j.out = None
                        finished.append(j)
                    used -= L.bytes
                    slots -= len(L.jobs)
                    self._events.append(L.event)
                    self._pinned.extend(L.pinned)
                    for a in L.arena:
                        self._arena_free(a)
                else:
                    still.append(L)
            inflight = still
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            admit = []
            while (waiting and slots + len(admit) < self.max_slots and len(admit) < self.max_batch
                   and len(inflight) < len(self.streams)):
                j = waiting[0]
                b = self.job_bytes(j)
                if used + b > self.budget and (used > 0 or admit):
                    break
                waiting.popleft()
                j.admitted = now
                used += b
                admit.append(j)
            if admit:
                slots += len(admit)
                inflight.append(self._launch(admit, self.streams[k % len(self.streams)]))
                k += 1
            elif not inflight and pending and not waiting:
                gap = pending[0].arrival - (time.perf_counter() - t0)
                if gap > 0:
                    time.sleep(min(gap, 0.001))
        torch.cuda.synchronize()
        return finished


def percentile(vals, q):
    vals = sorted(vals)
    if not vals:
        return float("nan")
    i = min(len(vals) - 1, max(0, int(round(q / 100.0 * (len(vals) - 1)))))
    return vals[i]


def summarize(jobs):
    lat = [j.done - j.arrival for j in jobs]
    elems = sum(j.n for j in jobs)
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return {"jobs": len(jobs), "elements": elems, "p50_ms": round(percentile(lat, 50) * 1e3, 4),
            "p99_ms": round(percentile(lat, 99) * 1e3, 4), "mean_ms": round(sum(lat) / len(lat) * 1e3, 4),
            "gelem_s": round(elems / span / 1e9, 4), "span_s": round(span, 4)}
