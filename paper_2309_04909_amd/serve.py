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


@dataclass
class Launch:
    event: torch.cuda.Event
    jobs: list
    batches: list = field(default_factory=list)
    records: list = field(default_factory=list)   # kept alive until the launch has completed
    bytes: int = 0


class Server:
    def __init__(self, pools, params, seeds: B.Seeds, hbm_budget: int, max_slots: int = 256, nstreams: int = 4,
                 keep_outputs: bool = False, rand_budget: int = 0):
        """pools[ell] = (x0, x1) device share pools; params[ell] = B.Params of that ring;
        rand_budget = HBM bytes for resident randomness records (0 = none)."""
        self.rand_budget = rand_budget
        self.pools = pools
        self.params = params
        self.seeds = seeds
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.keep = keep_outputs

    def warmup(self):
        """One small call per ring, op and lane-group size, so that no job pays
        for loading a kernel's code object on its first launch."""
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

    def _launch(self, jobs, stream):
        ev = torch.cuda.Event(enable_timing=True)
        L = Launch(ev, jobs)
        with torch.cuda.stream(stream):
            by_ell = {}
            for j in jobs:
                x0, x1 = self.pools[j.ell]
                j.y0 = torch.empty(j.n, dtype=x0.dtype, device=x0.device)
                j.y1 = torch.empty(j.n, dtype=x1.dtype, device=x1.device)
                L.bytes += self.job_bytes(j)
                seg = BT.Segment(x0[j.offset:j.offset + j.n], x1[j.offset:j.offset + j.n], j.y0, j.y1, op=j.op,
                                 nonce=j.nonce, elem_base=0, k_in=j.k_in, rand=j.rand)
                if j.rand is not None:               # released with the launch, once it has completed
                    L.records.append(j.rand)
                    j.rand = None
                by_ell.setdefault(j.ell, []).append(seg)
            for ell, segs in by_ell.items():
                prm = self.params[ell]
                if len(segs) == 1 and not (segs[0].rand is not None and segs[0].k_in):
                    self._single(segs[0], prm, stream)       # one job: the plain call needs no plan
                    continue
                rb = BT.RaggedBatch(prm, self.seeds, segs)
                rb.run(stream)
                L.batches.append(rb)
            ev.record(stream)
        return L

    def _single(self, sg, prm, stream):
        out = (sg.y0, sg.y1)
        relu = sg.op == B.BC_OP_RELU
        if sg.rand is not None:                      # online kernel on the resident record
            fn = B.relu_pre if relu else B.drelu_pre
            fn(sg.x0, sg.x1, prm, sg.rand, out=out, stream=stream)
        elif sg.k_in:
            fn = B.trunc_relu if relu else B.trunc_drelu
            fn(sg.x0, sg.x1, prm.ell + sg.k_in, sg.k_in, prm, self._seeds(sg.nonce), elem_base=sg.elem_base, out=out,
               stream=stream)
        else:
            fn = B.relu if relu else B.drelu
            fn(sg.x0, sg.x1, prm, self._seeds(sg.nonce), elem_base=sg.elem_base, out=out, stream=stream)

    def run(self, jobs):
        """Serve `jobs` (arrival times relative to the start); returns them with
        completion times filled in."""
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
                        if not self.keep:
                            j.y0 = j.y1 = None
                        finished.append(j)
                    used -= L.bytes
                    slots -= len(L.jobs)
                else:
                    still.append(L)
            inflight = still
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            admit = []
            while waiting and slots + len(admit) < self.max_slots and len(inflight) < len(self.streams):
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
