"""Ragged batches: many DReLU/ReLU share pairs in one persistent launch.

A batch shares one setting (ring, window, prime) and the three seeds; each
segment has its own length, op, nonce, global element offset and input
truncation k_in, and gets exactly the result of a single bc_drelu / bc_relu
(or, with k_in > 0, bc_trunc_drelu / bc_trunc_relu) call on it: the
truncate-then-ReLU of a whole layer chain is one launch.  The plan is
built on the host by the C ABI (bc_batch_plan), copied to device memory once,
and every run is a single kernel launch (bc_batch_run) that a HIP graph can
capture.
"""

import ctypes
from dataclasses import dataclass

import torch

from . import bicop as B


@dataclass
class Segment:
    x0: torch.Tensor
    x1: torch.Tensor
    y0: torch.Tensor
    y1: torch.Tensor
    op: int = B.BC_OP_RELU
    nonce: int = 0
    elem_base: int = 0
    k_in: int = 0          # truncate the inputs by k_in bits first (Alg. 5): shares of Z_2^(ell + k_in)
    rand: torch.Tensor = None   # precomputed randomness record (bicop.rand_expand), or None: draws from the seeds


def _records(params: B.Params, segments):
    width = B.ring_width(params.ell)
    recs = (B._Segment * len(segments))()
    m = (1 << 64) - 1
    for i, s in enumerate(segments):
        B._check_shares(s.x0, s.x1, width)
        B._check_shares(s.y0, s.y1, width, "outputs")
        if s.x0.numel() != s.y0.numel():
            raise ValueError("segment input and output lengths differ")
        rp, rd = (s.rand.data_ptr(), ctypes.pointer(B.rand_desc(s.rand))) if s.rand is not None else (None, None)
        recs[i] = B._Segment(s.x0.data_ptr(), s.x1.data_ptr(), s.y0.data_ptr(), s.y1.data_ptr(), s.x0.numel(),
                             s.elem_base, s.nonce & m, s.op, s.k_in, rp, rd)
    return recs


class RaggedBatch:
    def __init__(self, params: B.Params, seeds: B.Seeds, segments, tile_elems: int = 0, grid: int = 0):
        self.segments = list(segments)
        self._build(params, seeds, _records(params, self.segments), len(self.segments),
                    self.segments[0].x0.device, sum(s.x0.numel() for s in self.segments), tile_elems, grid)

    @classmethod
    def from_records(cls, params: B.Params, seeds: B.Seeds, records, device, elements: int, tile_elems: int = 0,
                     grid: int = 0, host_plan: torch.Tensor = None, dev_plan: torch.Tensor = None):
        """A batch from a ready array of bicop._Segment records (raw device
        pointers of contiguous share arrays of the ring's width on `device`,
        which the caller vouches for; the C ABI still checks every record).
        Serving builds its launches this way, without a tensor per segment,
        and passes buffers of its own to build the plan in: a pinned byte
        buffer and a device byte buffer of at least plan_bytes(n) bytes, which
        must outlive the run (a device allocation can wait for the whole
        device, so a loop that overlaps launches makes none per launch)."""
        self = cls.__new__(cls)
        self.segments = []
        self._build(params, seeds, records, len(records), device, elements, tile_elems, grid, host_plan, dev_plan)
        return self

    @staticmethod
    def plan_bytes(nseg: int) -> int:
        return int(B.lib.bc_batch_plan_bytes(nseg))

    def _build(self, params, seeds, recs, nseg, device, elements, tile_elems, grid, host_plan=None, dev_plan=None):
        self.params = params
        self.seeds = seeds
        if tile_elems == 0:                          # autotuned tile size, else the library default
            tile_elems = int(B.SCHEDULES.get("batch_tile", 0))
        self.grid = grid
        self.device = device
        nbytes = self.plan_bytes(nseg)
        # The plan is built in pinned host memory and uploaded asynchronously
        # on the current stream (runs on that stream, or on streams ordered
        # after it, see it); the host copy stays alive with this object.
        if host_plan is not None:
            if not host_plan.is_pinned() or host_plan.dtype != torch.uint8 or host_plan.numel() < nbytes:
                raise ValueError("host_plan must be a pinned uint8 buffer of at least plan_bytes(n) bytes")
            self.host_plan = host_plan[:nbytes]
        else:
            self.host_plan = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        B._check(B.lib.bc_batch_plan(recs, nseg, ctypes.byref(params.c()), tile_elems, self.host_plan.data_ptr(),
                                     nbytes), "batch_plan")
        if dev_plan is not None:
            if dev_plan.dtype != torch.uint8 or dev_plan.device != torch.device(device) or dev_plan.numel() < nbytes:
                raise ValueError("dev_plan must be a uint8 buffer on the batch's device of at least plan_bytes(n) bytes")
            self.dev_plan = dev_plan[:nbytes]
            self.dev_plan.copy_(self.host_plan, non_blocking=True)
        else:
            self.dev_plan = self.host_plan.to(device, non_blocking=True)
        self._c_seeds = seeds.c()
        self.elements = elements

    def run(self, stream=None):
        """Enqueue the one persistent launch on `stream` (default: current)."""
        B._check(B.lib.bc_batch_run(self.dev_plan.data_ptr(), self.host_plan.data_ptr(),
                                    ctypes.byref(self._c_seeds), self.grid, B._stream(stream, self.dev_plan)), "batch_run")

    def run_static(self, stream=None):
        """Enqueue the batch through bc_batch_run_static on `stream` (default:
        current): the plan goes into the library's fixed device area and
        nothing is allocated.  Calls that overlap on one GPU race for that
        area; calls on one stream are ordered."""
        B._check(B.lib.bc_batch_run_static(self.host_plan.data_ptr(), ctypes.byref(self._c_seeds), self.grid,
                                           B._stream(stream, self.dev_plan)), "batch_run_static")

    def capture(self):
        """Capture run() into a CUDA/HIP graph; returns the torch.cuda.CUDAGraph.

        The graph's kernel reads this batch's device plan, so the graph keeps
        the batch (and with it the plan) alive for as long as it exists."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        g.ragged_batch = self
        return g
