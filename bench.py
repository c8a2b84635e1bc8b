#!/usr/bin/env python3
"""Benchmark of the Bicoptor 2.0 DReLU/ReLU hot path on one MI355X.

One step is one pass of the key-bit workload: the 13-bit deterministic
truncation (Alg. 5) of 2^24 shared products z = x1 * x2 in Z_{2^64} and the
key-bit DReLU (Alg. 7, l = 64, k_lo = 13, l_x = 18, p = 2^19 - 1) of 2^24
shared fixed-point values x (f = 13, |x| < 2^30).  The two are independent:
the HBM-bound truncation runs on a second stream beside the ALU-bound DReLU,
and a step ends when both have.  Inputs are seeded synthetic data, resident
in HBM before timing starts.  `value` is DReLU elements per second of the
whole step.

Printed as one JSON line (rank 0), with extra sections:
  kernels           per-kernel average durations (HIP events on the launch stream)
  roofline          the dominant kernel (the fused DReLU) against its ALU roofline
  cpu_baseline      the CPU oracle timed on a bounded sample of the same workload
  kernels_alone     the step's two kernels each on its own
  streaming         trunc_det, trunc_prob and mod_switch alone: GB/s and %HBM
  batched_vs_plain  ResNet-18 ragged ReLU: one persistent graph launch vs 17 launches
  layer_chain       truncate-then-ReLU of every ResNet-18 layer in one batch launch
  precomputed_randomness  offline seed expansion, online call on shares + record
  replicated_sharing      RSS DReLU / ReLU (Alg. drelu2) beside the 2-of-2 calls
  truncate_then_multiply  Alg. linear vs multiply-then-truncate: time and e1 counts
  parties_apart     the DReLU as one kernel per party with packed messages in HBM
  plain_drelu       l = 64 without key bits (l_x = 32), 65,536 elements: us per call
  serving           continuous-batching request loop: p50/p99 latency and Gelem/s
  matmul_relu       truncate-then-ReLU of a 4096 x 4096 . 4096 x 1024 product
  batch_sweep       latency floor to throughput plateau over batch sizes
  copy_reference    a plain copy: achievable HBM bandwidth, counter scaling

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from paper_2309_04909_amd.prof_summary import KERNELS, source_hash  # noqa: E402

METRIC = "DReLU Gelem/s (ℓ=64, key bits), batched vs plain, %HBM peak; p50/p99"
HBM_PEAK_GBS = 8000.0
# 32-bit vector ALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz (the rate at
# which simple 32-bit VALU instructions issue; fp32 vector 157.3 TFLOP/s counts
# an FMA as two flops).  VOP3-class instructions (64-bit shifts, 32x32->64
# multiplies, three-operand forms) issue at half this rate.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12

KEYBIT = dict(ell=64, lx=18, k_lo=13, trunc_k=13, n=1 << 24, seed=2)
SIDE_TRUNC_BPC = 1          # blocks per CU of the truncation that overlaps the DReLU in a step
HEADLINE_WARM_S = 2.0       # the headline's warm-up lasts at least this long (clock ramp after the CPU leg)
SEEDS = (0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0)


# ------------------------------------------------------------- ALU op model


def shuffle_blocks(n: int) -> int:
    """Philox blocks of an element's shuffle: its n digits (the flip t of radix
    2, then the Fisher-Yates choices of radices 2..n) go to 64-bit chunks while
    the product of a chunk's radices stays <= 2^32, two chunks to a block."""
    chunks, prod = 1, 1
    for m in [2] + list(range(2, n + 1)):
        if prod * m > 1 << 32:
            chunks, prod = chunks + 1, 1
        prod *= m
    return (chunks + 1) // 2


PHILOX_OPS = 60          # 10 rounds x (two 32x32->64 multiplies + four XORs)
SLOT_OPS = 40            # per slot: two windows, adjacent sums, mod switch, two draws,
                         # two masked products with reshare, P2's sum and zero test
SLOT_OPS_WIDE = 64       # same with 64-bit field elements (l_x = 32)
DIGIT_OPS = 6            # per shuffle digit: two 32-bit multiplies and a carry add to cut it,
                         # then the Fisher-Yates step's read and two writes
TAIL_OPS = {"drelu": 12, "relu": 40,
            # replicated sharing at l = 64: [t], [s], the zero sharing, the product [s][t]
            # (two 64-bit multiplies per share), [s xor t], the finish; the ReLU adds a product
            "rss_drelu": 100, "rss_relu": 160}
# Philox blocks per element beyond the shuffle and the masks
TAIL_BLOCKS = {"drelu": 1, "relu": 3, "rss_drelu": 6, "rss_relu": 7}


def mask_blocks(n: int) -> int:
    """Philox blocks of an element's masks and reshares with the default prime:
    N-bit fields of one bit stream for N >= 17 (2N fields of N bits), else
    two slots to a block (32-bit words)."""
    if n >= 17:
        return -(-2 * n * n // 128)
    return (n + 1) // 2


def alg_ops_per_elem(op: str, lx: int) -> int:
    """32-bit integer operations per element of the fused kernel: 60 per Philox
    block, a fixed count per slot and per shuffle digit, and a per-op tail (the
    method's work, as a GEMM's flops count 2mnk)."""
    n = lx + 1
    wide = lx == 32
    blocks = shuffle_blocks(n) + mask_blocks(n) + TAIL_BLOCKS[op]
    return blocks * PHILOX_OPS + n * ((SLOT_OPS_WIDE if wide else SLOT_OPS) + DIGIT_OPS) + TAIL_OPS[op]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None if the
    kernel's code changed since the counters were taken."""
    src_hash = source_hash(KERNELS[kernel][1])
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f).get(kernel)
    if not t or t.get("source_hash") != src_hash:
        return None
    return t.get("bytes_per_launch")


# --------------------------------------------------------------- CPU oracle


def _oracle_chunk(args):
    from oracle import protocols as OPR
    x0, x1, z0, z1, g, p = args
    c = KEYBIT
    OPR.trunc_det(z0, z1, c["ell"], c["trunc_k"], 0)
    OPR.drelu(x0, x1, c["ell"], c["lx"], c["k_lo"], p, SEEDS, 7, g=g)
    return len(g)


def cpu_baseline(inputs, sample: int, workers: int):
    """The oracle (as it stands) on the first `sample` elements of the step's inputs,
    over `workers` forked processes.  Runs before the GPU is touched."""
    import multiprocessing as mp
    from oracle.params import default_prime
    x0, x1, z0, z1 = inputs
    p = default_prime(KEYBIT["lx"])
    chunks = np.array_split(np.arange(sample, dtype=np.uint64), workers * 4)
    jobs = [(x0[c[0]:c[-1] + 1], x1[c[0]:c[-1] + 1], z0[c[0]:c[-1] + 1], z1[c[0]:c[-1] + 1], c, p)
            for c in chunks if len(c)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        done = sum(pool.map(_oracle_chunk, jobs))
    dt = time.perf_counter() - t0
    # the same oracle in this one process on the first chunks (about 2^20 elements)
    single = []
    for j in jobs:
        single.append(j)
        if sum(len(c[4]) for c in single) >= (1 << 20):
            break
    t1 = time.perf_counter()
    done1 = sum(_oracle_chunk(j) for j in single)
    dt1 = time.perf_counter() - t1
    return {"value": done / dt / 1e9, "unit": "Gelem/s", "cores": workers, "kind": "oracle",
            "sample": f"first {done} elements of the step (13-bit trunc_det of z and key-bit DReLU of x), "
                      f"{workers} processes, {dt:.1f} s wall",
            "single_process": {"value": done1 / dt1 / 1e9, "unit": "Gelem/s", "elements": done1,
                               "seconds": round(dt1, 2)},
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------- GPU parts


HIP_EVENT_DISABLE_SYSTEM_FENCE = 0x20000000      # hipEventCreateWithFlags flags (hip_runtime_api.h)
HIP_EVENT_DISABLE_TIMING = 0x2


def _hip_runtime():
    """The HIP runtime this process already has loaded (torch's, which the
    library resolves to as well), or None if there is not exactly one."""
    import ctypes
    try:
        with open("/proc/self/maps") as f:
            paths = sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return None
    if len(paths) != 1:
        return None
    hip = ctypes.CDLL(paths[0])
    hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
    hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    hip.hipStreamWaitEvent.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint]
    return hip


class Timer:
    """HIP events on the stream a kernel is launched on (default: torch's
    current stream), created with hipEventDisableSystemFence: they only time,
    so recording them skips the system-scope cache writeback that a default
    event does, which would also slow the launch after it.  Falls back to
    torch's events if the runtime cannot be found."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}
        self.hip = _hip_runtime()
        self.kind = "HIP events without the system-scope fence" if self.hip else "torch.cuda.Event"

    def _record(self, stream):
        if self.hip is None:
            e = self.torch.cuda.Event(enable_timing=True)
            e.record(stream)
            return e
        import ctypes
        e = ctypes.c_void_p()
        rc = self.hip.hipEventCreateWithFlags(ctypes.byref(e), HIP_EVENT_DISABLE_SYSTEM_FENCE)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
        st = stream if stream is not None else self.torch.cuda.current_stream()
        rc = self.hip.hipEventRecord(e, st.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")
        return e

    def start(self, stream=None):
        return self._record(stream)

    def stop(self, name, s, stream=None):
        self.pairs.setdefault(name, []).append((s, self._record(stream)))

    def avg_ms(self, name):
        """Mean duration; call after the device has synchronised."""
        ps = self.pairs.get(name, [])
        if self.hip is None:
            return sum(s.elapsed_time(e) for s, e in ps) / max(1, len(ps))
        import ctypes
        tot = 0.0
        for s, e in ps:
            ms = ctypes.c_float()
            rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), s, e)
            if rc != 0:
                raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
            tot += ms.value
        return tot / max(1, len(ps))

    def release(self):
        if self.hip is not None:
            for ps in self.pairs.values():
                for s, e in ps:
                    self.hip.hipEventDestroy(s)
                    self.hip.hipEventDestroy(e)
        self.pairs = {}


class StreamJoins:
    """Cross-stream waits of the two-stream step: a HIP event recorded on the
    producing stream and waited on by the other, created without timing and
    without the system-scope fence (both streams are on one device and
    nothing on the host reads the data).  One event serves every join: a
    wait takes the event's state when it is enqueued, so recording it again
    for the next join leaves earlier waits alone.  Falls back to torch's
    wait_stream if the runtime cannot be found."""

    def __init__(self, torch):
        import ctypes
        self.hip = _hip_runtime()
        self.event = None
        self.kind = "HIP events without timing or the system-scope fence" if self.hip else "torch wait_stream"
        if self.hip is not None:
            e = ctypes.c_void_p()
            rc = self.hip.hipEventCreateWithFlags(ctypes.byref(e), HIP_EVENT_DISABLE_SYSTEM_FENCE |
                                                  HIP_EVENT_DISABLE_TIMING)
            if rc != 0:
                raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
            self.event = e

    def wait(self, dst, src):
        """dst waits for the work enqueued on src so far."""
        if self.hip is None:
            dst.wait_stream(src)
            return
        import ctypes
        rc = self.hip.hipEventRecord(self.event, ctypes.c_void_p(src.cuda_stream))
        if rc == 0:
            rc = self.hip.hipStreamWaitEvent(ctypes.c_void_p(dst.cuda_stream), self.event, 0)
        if rc != 0:
            raise RuntimeError(f"stream join failed ({rc})")

    def release(self):
        if self.event is not None:
            self.hip.hipEventDestroy(self.event)
        self.event = None


def to_dev(torch, a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()


def run_keybit(torch, B, inputs, steps, warmup):
    c = KEYBIT
    x0, x1, z0, z1 = (to_dev(torch, a) for a in inputs)
    # the key-bit window of Sec. 6.1 for |x| < 2^30 at f = 13 fractional bits
    prm = B.keybit_params(c["ell"], 13, B.keybit_int_bits(1 << 30, 13), 0)
    assert (prm.lx, prm.k_lo) == (c["lx"], c["k_lo"]), prm
    sd = B.Seeds(*SEEDS, 7)
    y0, y1 = torch.empty_like(x0), torch.empty_like(x1)
    t0, t1 = torch.empty_like(z0), torch.empty_like(z1)

    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()                     # default priority
    joins = StreamJoins(torch)

    def step(timer=None):
        joins.wait(side, main)                      # the step starts on both streams together
        s = timer.start(side) if timer else None
        B.trunc_det(z0, z1, c["ell"], c["trunc_k"], 0, out=(t0, t1), stream=side)
        if timer:
            timer.stop("trunc_det", s, side)
        s = timer.start() if timer else None
        B.drelu(x0, x1, prm, sd, out=(y0, y1))
        if timer:
            timer.stop("drelu", s)
        joins.wait(main, side)                      # and ends when both are done

    # The truncation beside the DReLU runs on one block per compute unit: it
    # needs well under 1 TB/s to finish inside the DReLU, and a narrow grid
    # leaves the ALU-bound DReLU's issue slots alone (a step measured 0.653 ms
    # against 0.674 ms with the standalone schedule of 64 blocks per CU).
    standalone_bpc = B.get_schedule("stream", 0, 8)
    B.set_schedule("stream", 0, SIDE_TRUNC_BPC, 8)
    try:
        # Warm-up: at least `warmup` steps and at least HEADLINE_WARM_S seconds
        # of them.  The GPU sits idle while the CPU leg runs before this, and
        # its clock takes longer to ramp back up than a few steps last.  The
        # queue is drained every 64 steps so that the time is device time.
        t_warm = time.perf_counter()
        warm_steps = 0
        while warm_steps < warmup or time.perf_counter() - t_warm < HEADLINE_WARM_S:
            step()
            warm_steps += 1
            if warm_steps % 64 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        warm_s = time.perf_counter() - t_warm
        # the timed region: barrier (single GPU: none) + synchronize on both
        # sides; HIP events between the kernels give their durations
        timer = Timer(torch)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            step(timer)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
    finally:
        B.set_schedule("stream", 0, standalone_bpc, 8)
        joins.release()
    times = {"trunc_det": timer.avg_ms("trunc_det"), "drelu": timer.avg_ms("drelu"), "events": timer.kind,
             "joins": joins.kind, "warmup_s": warm_s, "warmup_steps_run": warm_steps}
    timer.release()
    return wall, times


def run_alone(torch, B, inputs, steps, warmup):
    """The step's two kernels each alone (one stream, the standalone schedule)."""
    c = KEYBIT
    x0, x1, z0, z1 = (to_dev(torch, a) for a in inputs)
    prm, sd = B.Params(c["ell"], c["lx"], c["k_lo"]), B.Seeds(*SEEDS, 7)
    y0, y1, t0, t1 = (torch.empty_like(a) for a in (x0, x1, z0, z1))
    td = _event_ms(torch, lambda: B.trunc_det(z0, z1, c["ell"], c["trunc_k"], 0, out=(t0, t1)), steps, warmup)
    dr = _event_ms(torch, lambda: B.drelu(x0, x1, prm, sd, out=(y0, y1)), steps, warmup)
    gbs = 32 * c["n"] / (td * 1e-3) / 1e9
    return {"drelu_ms": round(dr, 4), "drelu_gelem_s": round(c["n"] / dr / 1e6, 3), "trunc_det_ms": round(td, 4),
            "trunc_det_gbs": round(gbs, 1), "trunc_det_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def _batched_vs_plain(torch, B, steps, warmup, batch):
    """The 17 ReLU activation tensors of a ResNet-18 pass at `batch`, 224x224:
    one persistent launch replayed from a HIP graph against 17 plain launches,
    called one by one and captured into a graph of their own."""
    from paper_2309_04909_amd import batch as BT
    prm = B.Params(64, 7, 11)
    seeds = SEEDS
    data = W.resnet18_relu(seed=4, batch=batch)
    segs = []
    for i, (_, (x0, x1)) in enumerate(data):
        d0, d1 = to_dev(torch, x0), to_dev(torch, x1)
        segs.append(BT.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=B.BC_OP_RELU, nonce=100 + i))
    del data
    total = sum(s.x0.numel() for s in segs)
    rb = BT.RaggedBatch(prm, B.Seeds(*seeds), segs)
    graph = rb.capture()
    sds = [B.Seeds(*seeds, s.nonce) for s in segs]

    def plain():
        for s, sd in zip(segs, sds):
            B.relu(s.x0, s.x1, prm, sd, out=(s.y0, s.y1))

    plain()
    torch.cuda.synchronize()
    ref = [(s.y0.clone(), s.y1.clone()) for s in segs]
    side = torch.cuda.Stream()                    # the 17 plain launches captured as one graph
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plain()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    plain_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(plain_graph):
        plain()

    ms_plain = _event_ms(torch, plain, steps, warmup)
    ms_plain_graph = _event_ms(torch, plain_graph.replay, steps, warmup)
    same = all(torch.equal(a, s.y0) and torch.equal(b, s.y1) for (a, b), s in zip(ref, segs))
    ms_batch = _event_ms(torch, graph.replay, steps, warmup)
    same &= all(torch.equal(a, s.y0) and torch.equal(b, s.y1) for (a, b), s in zip(ref, segs))
    return {"workload": f"ResNet-18 ReLU activations, batch {batch}, 224x224: 17 tensors, {total} elements, "
                        "l=64, k_lo=11, l_x=7 (p=251)",
            "elements": total, "plain_ms": round(ms_plain, 4), "plain_graph_ms": round(ms_plain_graph, 4),
            "batched_ms": round(ms_batch, 4), "plain_gelem_s": round(total / ms_plain / 1e6, 3),
            "batched_gelem_s": round(total / ms_batch / 1e6, 3), "speedup": round(ms_plain / ms_batch, 4),
            "speedup_vs_plain_graph": round(ms_plain_graph / ms_batch, 4), "identical_outputs": bool(same),
            "batched": "one persistent launch (bc_batch_run) replayed from a HIP graph",
            "plain": "17 bc_relu launches", "plain_graph": "the 17 bc_relu launches captured in one HIP graph"}


def run_batched_vs_plain(torch, B, steps, warmup):
    """Batched against per-layer plain launches at batch 32 (large segments,
    the configured workload) and at batch 1 (17 segments of 1,568 to 802,816
    elements, where launch and tail costs show)."""
    out = _batched_vs_plain(torch, B, steps, warmup, 32)
    out["batch1"] = _batched_vs_plain(torch, B, max(steps, 50), max(warmup, 10), 1)
    return out


def run_chain(torch, B, steps, warmup, batch=32):
    """Truncate-then-ReLU over a whole layer chain: the 17 ResNet-18 ReLU
    tensors (batch 32) arrive as products with 26 fractional bits in Z_2^64;
    each is truncated by 13 bits (Alg. 5) into Z_2^51 and ReLU'd (k_lo = 11,
    l_x = 7).  One graph-replayed batch launch with per-segment truncation
    against 17 fused calls and against 34 two-pass calls (trunc_det, relu)."""
    from paper_2309_04909_amd import batch as BT
    prm = B.Params(51, 7, 11)
    data = W.resnet18_relu(seed=4, batch=batch, f=26)
    segs = []
    for i, (_, (x0, x1)) in enumerate(data):
        d0, d1 = to_dev(torch, x0), to_dev(torch, x1)
        segs.append(BT.Segment(d0, d1, torch.empty_like(d0), torch.empty_like(d1), op=B.BC_OP_RELU, nonce=200 + i,
                               k_in=13))
    del data
    total = sum(s.x0.numel() for s in segs)
    rb = BT.RaggedBatch(prm, B.Seeds(*SEEDS), segs)
    graph = rb.capture()
    tmp = [(torch.empty_like(s.x0), torch.empty_like(s.x1)) for s in segs]
    outs = [(torch.empty_like(s.x0), torch.empty_like(s.x1)) for s in segs]

    def fused():
        for s, o in zip(segs, outs):
            B.trunc_relu(s.x0, s.x1, 64, 13, prm, B.Seeds(*SEEDS, s.nonce), out=o)

    def two_pass():
        for s, t, o in zip(segs, tmp, outs):
            B.trunc_det(s.x0, s.x1, 64, 13, 0, out=t)
            B.relu(t[0], t[1], prm, B.Seeds(*SEEDS, s.nonce), out=o)

    # precomputed randomness: every segment's draws expanded offline into a
    # resident record; the same chain then runs as one batch launch of the
    # online element (shares and records streamed, no PRG)
    rsegs = [BT.Segment(s.x0, s.x1, torch.empty_like(s.x0), torch.empty_like(s.x1), op=s.op, nonce=s.nonce, k_in=13)
             for s in segs]

    def expand():
        for s, r in zip(segs, rsegs):
            r.rand = B.rand_expand(B.BC_OP_RELU, prm, B.Seeds(*SEEDS, s.nonce), s.x0.numel(), out=r.rand)

    expand()
    rec_bytes = sum(r.rand.numel() for r in rsegs)
    rgraph = BT.RaggedBatch(prm, B.Seeds(*SEEDS), rsegs).capture()

    # the variants interleaved over three rounds, best of each (the first
    # timings after the host-side setup run on a GPU that is still clocking up)
    ms_batch = ms_fused = ms_two = ms_online = ms_offline = float("inf")
    same_fused = same_two = same_online = True
    for _ in range(3):
        ms_batch = min(ms_batch, _event_ms(torch, graph.replay, steps, warmup))
        ms_online = min(ms_online, _event_ms(torch, rgraph.replay, steps, warmup))
        same_online &= all(torch.equal(r.y0, s.y0) and torch.equal(r.y1, s.y1) for s, r in zip(segs, rsegs))
        ms_offline = min(ms_offline, _event_ms(torch, expand, 2, 1))
        ms_fused = min(ms_fused, _event_ms(torch, fused, steps, warmup))
        same_fused &= all(torch.equal(o[0], s.y0) and torch.equal(o[1], s.y1) for s, o in zip(segs, outs))
        ms_two = min(ms_two, _event_ms(torch, two_pass, steps, warmup))
        same_two &= all(torch.equal(o[0], s.y0) and torch.equal(o[1], s.y1) for s, o in zip(segs, outs))
    online_bytes = 4 * 8 * total + rec_bytes            # shares in and out, plus the records
    return {"workload": f"ResNet-18 ReLU inputs as products (f = 26) in Z_2^64, batch {batch}: 17 tensors, {total} "
                        "elements; trunc_det by 13 into Z_2^51, then ReLU (k_lo = 11, l_x = 7, p = 251)",
            "elements": total, "batched_ms": round(ms_batch, 4), "fused_calls_ms": round(ms_fused, 4),
            "two_pass_ms": round(ms_two, 4), "batched_gelem_s": round(total / ms_batch / 1e6, 3),
            "online_batched_ms": round(ms_online, 4), "online_gelem_s": round(total / ms_online / 1e6, 3),
            "online_gbs": round(online_bytes / ms_online / 1e6, 1),
            "online_hbm_frac": round(online_bytes / ms_online / 1e6 / HBM_PEAK_GBS, 4),
            "record_bytes_per_elem": round(rec_bytes / total, 2), "offline_ms": round(ms_offline, 4),
            "identical_outputs": bool(same_fused and same_two and same_online),
            "batched": "one persistent launch with per-segment truncation, replayed from a HIP graph",
            "online_batched": "the same launch with every segment on its precomputed record (shuffle, masks and "
                              "P2's [c]_1; the parties regenerate their triple shares); bytes = 32 per element of "
                              "shares plus the records",
            "fused_calls": "17 bc_trunc_relu launches", "two_pass": "17 x (bc_trunc_det + bc_relu)"}


def run_plain_drelu(torch, B, steps, warmup):
    """l = 64 with no key-bit reduction: l_x = 32 (all windows of the 64-bit ring) and
    the paper's default l_x = 31, 65,536 elements (latency-bound)."""
    _, (x0, x1) = W.plain_drelu(seed=1)
    d0, d1 = to_dev(torch, x0), to_dev(torch, x1)
    y0, y1 = torch.empty_like(d0), torch.empty_like(d1)
    out = {"workload": "plain DReLU, l=64, 65,536 elements, v ~ U(-64, 64), f=13"}
    for lx in (32, 31):
        prm = B.Params(64, lx, 0)
        sd = B.Seeds(*SEEDS, 11)
        ms = _event_ms(torch, lambda: B.drelu(d0, d1, prm, sd, out=(y0, y1)), steps, warmup)
        out[f"lx{lx}_us_per_call"] = round(ms * 1e3, 2)
        out[f"lx{lx}_gelem_s"] = round(d0.numel() / ms / 1e6, 3)
    return out


SERVE_PARAMS = {64: (64, 18, 13), 32: (32, 8, 8)}
POOL_LOG2 = 24


def serving_jobs(S, rng_seed, rate, count, pool_n):
    """Seeded Poisson jobs (sizes log-uniform in [2^10, 2^24], op and ring 50/50);
    rate = None puts every arrival at t = 0 (saturation)."""
    rng = np.random.default_rng(rng_seed)
    arr = W.serving_arrivals(rng_seed, rate or 1.0, count)
    jobs = []
    for i, (t, n, op, ell) in enumerate(arr):
        off = int(rng.integers(0, pool_n - n + 1))
        jobs.append(S.Job(i, t if rate else 0.0, n, 0 if op == "drelu" else 1, ell, off, 0x5E5E0000 + i))
    return jobs


def run_serving(torch, B, count=600):
    """Continuous batching under Poisson load at 0.3/0.6/0.9 of the saturated rate."""
    from paper_2309_04909_amd import serve as S
    pool_n = 1 << POOL_LOG2
    pools = {}
    for ell in (64, 32):
        _, (x0, x1) = W.serving_values(100 + ell, pool_n, ell)
        pools[ell] = (to_dev(torch, x0), to_dev(torch, x1))
    params = {ell: B.Params(*SERVE_PARAMS[ell]) for ell in (64, 32)}
    seeds = B.Seeds(*SEEDS)
    budget = 64 << 30
    srv = S.Server(pools, params, seeds, hbm_budget=budget, max_slots=256, nstreams=4)
    srv.warmup()
    srv.run(serving_jobs(S, 7, None, 50, pool_n))                         # warm-up
    sat = S.summarize(srv.run(serving_jobs(S, 8, None, count, pool_n)))
    mean_n = (2.0 ** 24 - 2.0 ** 10) / (14 * np.log(2.0))
    out = {"workload": f"{count} jobs per rate, sizes log-uniform [2^10, 2^24], DReLU/ReLU 50/50, "
                       "l in {32, 64} 50/50 (l=64: k_lo=13, l_x=18; l=32: k_lo=8, l_x=8), "
                       "inputs resident in HBM, 64 GiB admission budget, 4 streams",
           "saturated": sat}
    for frac in (0.3, 0.6, 0.9):
        rate = frac * sat["gelem_s"] * 1e9 / mean_n
        res = S.summarize(srv.run(serving_jobs(S, 9 + int(frac * 10), rate, count, pool_n)))
        res["offered_jobs_per_s"] = round(rate, 1)
        out[f"load_{frac}"] = res
    # the 0.6 load again, with randomness records expanded offline and resident
    # (a 32 GiB budget, filled in arrival order): those jobs run the online kernel
    rate = 0.6 * sat["gelem_s"] * 1e9 / mean_n
    jobs = serving_jobs(S, 15, rate, count, pool_n)
    srv_pre = S.Server(pools, params, seeds, hbm_budget=budget, max_slots=256, nstreams=4, rand_budget=32 << 30)
    with_rec, rec_bytes, offline_s = srv_pre.prepare(jobs)
    res = S.summarize(srv_pre.run(jobs))
    res.update({"offered_jobs_per_s": round(rate, 1), "jobs_with_records": with_rec,
                "record_gib": round(rec_bytes / 2 ** 30, 2), "offline_s": round(offline_s, 3)})
    out["load_0.6_precomputed"] = res
    # the 0.6 load once more as layer-chain traffic: every third job is a
    # truncate-then-DReLU/ReLU step (products with 26 fractional bits in
    # Z_2^64, truncated by 13 bits into Z_2^51 inside the launch; k_lo = 11,
    # l_x = 7), with records resident as above
    _, (c0, c1) = W.chain_values(102, pool_n)
    cpools = dict(pools)
    cpools[51] = (to_dev(torch, c0), to_dev(torch, c1))
    cparams = dict(params)
    cparams[51] = B.Params(51, 7, 11)
    jobs = serving_jobs(S, 16, rate, count, pool_n)
    for j in jobs[::3]:
        j.ell, j.k_in = 51, 13
    srv_c = S.Server(cpools, cparams, seeds, hbm_budget=budget, max_slots=256, nstreams=4, rand_budget=32 << 30)
    srv_c.warmup()
    with_rec, rec_bytes, offline_s = srv_c.prepare(jobs)
    chain_rec = sum(1 for j in jobs if j.k_in and j.rand is not None)
    res = S.summarize(srv_c.run(jobs))
    res.update({"offered_jobs_per_s": round(rate, 1), "chain_jobs": len(jobs[::3]), "jobs_with_records": with_rec,
                "chain_jobs_with_records": chain_rec, "record_gib": round(rec_bytes / 2 ** 30, 2),
                "offline_s": round(offline_s, 3)})
    out["load_0.6_chain_precomputed"] = res
    return out


def run_matmul_relu(torch, B, steps, warmup):
    """ReLU after a fixed-point matmul: Z = A B (A 4096x4096, B 4096x1024, exact),
    shared, truncated by f bits (Alg. 5), then ReLU on all 4,194,304 outputs.
    Two-pass (trunc_det then relu) vs the fused bc_trunc_relu; l = 64 (f = 13)
    and the l = 32 variant (f = 8)."""
    out = {"workload": "ReLU after matmul [4096x4096].[4096x1024], 4,194,304 outputs"}
    for ell, f, lx, k_lo in ((64, 13, 11, 13), (32, 8, 7, 10)):
        _, (z0, z1) = W.matmul_relu(seed=3, ell=ell)
        d0, d1 = to_dev(torch, z0), to_dev(torch, z1)
        prm, sd = B.Params(ell - f, lx, k_lo), B.Seeds(*SEEDS, 21)
        t0, t1 = torch.empty_like(d0), torch.empty_like(d1)
        y0, y1 = torch.empty_like(d0), torch.empty_like(d1)

        def two_pass():
            B.trunc_det(d0, d1, ell, f, 0, out=(t0, t1))
            B.relu(t0, t1, prm, sd, out=(y0, y1))

        def fused():
            B.trunc_relu(d0, d1, ell, f, prm, sd, out=(y0, y1))

        res = {}
        for name, fn in (("two_pass", two_pass), ("fused", fused)):
            ms = _event_ms(torch, fn, steps, warmup)
            res[f"{name}_ms"] = round(ms, 4)
            res[f"{name}_gelem_s"] = round(d0.numel() / ms / 1e6, 3)
        out[f"l{ell}"] = dict(res, setting=f"trunc {f} -> Z_2^{ell - f}, k_lo={k_lo}, l_x={lx}")
    return out


# Tab. 6 / Tab. 7 (three P100 servers, LAN1): microseconds per DReLU / ReLU batch
PAPER_LAN1_US = {"drelu": {1: 932.05, 1000: 997.36, 10000: 1375.86, 100000: 5698.69, 1000000: 58608.3},
                 "relu": {1: 1519.43, 1000: 1608.76, 10000: 2275.01, 100000: 9958.73, 1000000: 90185.9}}


def run_sweep(torch, B, steps, warmup):
    """Batch sizes of the paper's unit experiments (1 ... 10^6) at l = 64, l_x = 7
    (k_lo = 11): microseconds per call on one GPU, next to the paper's LAN1 times
    (three networked P100 servers, where the network dominates: context only)."""
    n_max = 10 ** 6
    rng = np.random.default_rng(12)
    x = W.encode(W.fixed_point(rng.standard_normal(n_max), 13), 64)
    x0, x1 = W.share(x, 64, rng)
    d0, d1 = to_dev(torch, x0), to_dev(torch, x1)
    y0, y1 = torch.empty_like(d0), torch.empty_like(d1)
    prm, sd = B.Params(64, 7, 11), B.Seeds(*SEEDS, 5)
    out = {"workload": "DReLU / ReLU, l=64, k_lo=11, l_x=7, N(0,1) 2^13 values; paper = Tab. 6/7 LAN1 (context)"}
    for op, fn in (("drelu", B.drelu), ("relu", B.relu)):
        rows = {}
        for n in (1, 1000, 10000, 100000, 1000000):
            a0, a1, b0, b1 = d0[:n], d1[:n], y0[:n], y1[:n]
            us = _event_ms(torch, lambda: fn(a0, a1, prm, sd, out=(b0, b1)), steps, warmup) * 1e3
            rows[str(n)] = {"us": round(us, 2), "gelem_s": round(n / us / 1e3, 4), "paper_lan1_us": PAPER_LAN1_US[op][n]}
        out[op] = rows
    return out


def _event_ms(torch, fn, steps, warmup, warm_s=0.03):
    """Average milliseconds per call of fn over `steps` calls, timed with HIP
    events on the current stream, after at least `warmup` calls and warm_s
    seconds of untimed calls (a section's first timing otherwise catches the
    GPU still clocking up after the host-side setup)."""
    t0 = time.perf_counter()
    done = 0
    while done < warmup or time.perf_counter() - t0 < warm_s:
        fn()
        torch.cuda.synchronize()
        done += 1
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def run_precomputed(torch, B, inputs, steps, warmup):
    """Precomputed-randomness mode, labelled separately: the offline expansion of the
    seeds into the resident record (bc_rand_expand), the online call that streams
    shares plus record (bc_drelu_pre / bc_relu_pre), and the fused call beside them,
    on the key-bit inputs (2^24 elements, l = 64)."""
    x0, x1 = to_dev(torch, inputs[0]), to_dev(torch, inputs[1])
    n = x0.numel()
    out = {"workload": f"{n} key-bit inputs, l=64; offline = seed expansion into the record, online = "
                       "shares + record streamed, fused = in-kernel PRG"}
    sd = B.Seeds(*SEEDS, 21)
    for name, op, prm in (("drelu_lx18", B.BC_OP_DRELU, B.Params(64, 18, 13)),
                          ("relu_lx7", B.BC_OP_RELU, B.Params(64, 7, 11))):
        online = B.drelu_pre if op == B.BC_OP_DRELU else B.relu_pre
        fused = B.drelu if op == B.BC_OP_DRELU else B.relu
        rand = B.rand_expand(op, prm, sd, n)
        y0, y1 = torch.empty_like(x0), torch.empty_like(x1)
        f0, f1 = torch.empty_like(x0), torch.empty_like(x1)
        ms_off = _event_ms(torch, lambda: B.rand_expand(op, prm, sd, n, out=rand), steps, warmup)
        ms_on = _event_ms(torch, lambda: online(x0, x1, prm, rand, out=(y0, y1)), steps, warmup)
        ms_fu = _event_ms(torch, lambda: fused(x0, x1, prm, sd, out=(f0, f1)), steps, warmup)
        same = bool(torch.equal(y0, f0) and torch.equal(y1, f1))
        rb = B.rand_bytes(op, prm, n)
        byt = 32 * n + rb
        out[name] = {"record_bytes_per_elem": round(rb / n, 1), "offline_ms": round(ms_off, 4),
                     "online_ms": round(ms_on, 4), "fused_ms": round(ms_fu, 4),
                     "online_gelem_s": round(n / ms_on / 1e6, 3), "fused_gelem_s": round(n / ms_fu / 1e6, 3),
                     "online_gbs": round(byt / ms_on / 1e6, 1),
                     "online_hbm_frac": round(byt / ms_on / 1e6 / HBM_PEAK_GBS, 4),
                     "identical_to_fused": same}
        del rand
    return out


def run_rss(torch, B, inputs, steps, warmup):
    """Replicated-sharing DReLU / ReLU (Alg. drelu2) on the 2^24 key-bit values,
    shared as ([x]_0 - a, a, [x]_1) with a uniform, at the key-bit setting
    (l_x = 18) and at l_x = 7; the 2-of-2 call on the same values beside it."""
    x0, x1 = inputs[0], inputs[1]
    n = x0.size
    a = np.random.default_rng(31).integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2)
    xs = tuple(to_dev(torch, v) for v in (x0 - a, a, x1))
    u0, u1 = to_dev(torch, x0), to_dev(torch, x1)
    out = {"workload": f"{n} key-bit values in Z_2^64 as replicated shares; 48 B/elem algorithmic "
                       "(three shares in, three out)"}
    sd, sd2 = B.RssSeeds(*SEEDS, 0x5EED012, 0x5EED2, 41), B.Seeds(*SEEDS, 41)
    ys = tuple(torch.empty_like(v) for v in xs)
    y0, y1 = torch.empty_like(u0), torch.empty_like(u1)
    for name, prm in (("lx18", B.Params(64, 18, 13)), ("lx7", B.Params(64, 7, 11))):
        for op in ("drelu", "relu"):
            rss = B.rss_drelu if op == "drelu" else B.rss_relu
            ubl = B.drelu if op == "drelu" else B.relu
            ms = _event_ms(torch, lambda: rss(xs, prm, sd, out=ys), steps, warmup)
            ms_ubl = _event_ms(torch, lambda: ubl(u0, u1, prm, sd2, out=(y0, y1)), steps, warmup)
            ops = alg_ops_per_elem("rss_" + op, prm.lx)
            tops = ops * n / (ms * 1e-3) / 1e12
            out[f"{op}_{name}"] = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 3),
                                   "gbs": round(48 * n / ms / 1e6, 1),
                                   "hbm_frac": round(48 * n / ms / 1e6 / HBM_PEAK_GBS, 4),
                                   "ops_per_elem": ops, "alu_frac": round(tops / VALU_PEAK_TOPS, 4),
                                   "two_of_two_ms": round(ms_ubl, 4)}
    return out


def run_linear(torch, B, steps, warmup):
    """Alg. linear against multiply-then-truncate: the elementwise secure product
    of 2^24 pairs of 31-bit fixed-point values (5 + 26 bits, the l = 64 setting
    of Sec. 4) in Z_2^64, truncated by f = 26.  Times each order (48 B/elem
    algorithmic: four input shares, two output shares) and counts the elements
    whose result is off by more than 2^32 from floor(x y / 2^26): the e1 failures
    (an e1 adds about 2^(64-26); e0 and the truncate-first order's lost precision
    stay below 2^20)."""
    (x, (x0, x1)), (y, (y0, y1)) = W.linear_factors(seed=5)
    n = x.size
    d = [to_dev(torch, v) for v in (x0, x1, y0, y1)]
    z0, z1 = torch.empty_like(d[0]), torch.empty_like(d[1])
    sd = B.Seeds(*SEEDS, 77)
    xs, ys = W.signed_values(x, 64).astype(np.int64), W.signed_values(y, 64).astype(np.int64)
    exact = (xs * ys) >> 26
    rate = float(np.mean(np.abs(xs.astype(np.float64) * ys.astype(np.float64)))) / 2.0 ** 64
    out = {"workload": f"{n} products of 31-bit fixed-point factors (f = 26) in Z_2^64; 48 B/elem algorithmic",
           "expected_e1_rate_after": round(rate, 5)}
    for name, order, f in (("none", B.BC_TRUNC_NONE, 0), ("after", B.BC_TRUNC_AFTER, 26),
                           ("before", B.BC_TRUNC_BEFORE, 26)):
        ms = _event_ms(torch, lambda: B.mul_trunc(*d, 64, f, order, sd, out=(z0, z1)), steps, warmup)
        r = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2), "gbs": round(48 * n / ms / 1e6, 1),
             "hbm_frac": round(48 * n / ms / 1e6 / HBM_PEAK_GBS, 4)}
        if f:
            got = (z0.cpu().numpy().view(np.uint64) + z1.cpu().numpy().view(np.uint64)).view(np.int64)
            err = np.abs(got - exact)
            e1 = err > (1 << 32)
            r["e1_failures"] = int(np.count_nonzero(e1))
            r["max_error_without_e1"] = int(err[~e1].max())
        out[name] = r
    return out


def run_split(torch, B, inputs, steps, warmup):
    """The DReLU with the parties apart (each party's kernel on its own, the
    round-1 messages bit-packed in HBM as they would cross a link) on the 2^24
    key-bit values, beside the fused call.  Per kernel: time and HBM bytes
    (send: own share in, packed message out; reply: both messages in, two
    reply shares out; finish: reply share in, output share out)."""
    x0, x1 = to_dev(torch, inputs[0]), to_dev(torch, inputs[1])
    n = x0.numel()
    out = {"workload": f"{n} key-bit values, l = 64; messages word-major, ceil(N^2 / 32) words per element"}
    sd = B.Seeds(*SEEDS, 61)
    for name, prm in (("lx18", B.Params(64, 18, 13)), ("lx7", B.Params(64, 7, 11))):
        words = B.msg_words(prm.npos)
        m0 = torch.empty((words, n), dtype=torch.int32, device="cuda")
        m1 = torch.empty_like(m0)
        r0, r1, y0, y1 = (torch.empty_like(x0) for _ in range(4))
        ms = {
            "send_p0": _event_ms(torch, lambda: B.drelu_send(0, x0, prm, sd, out=m0), steps, warmup),
            "send_p1": _event_ms(torch, lambda: B.drelu_send(1, x1, prm, sd, out=m1), steps, warmup),
            "reply_p2": _event_ms(torch, lambda: B.drelu_reply(m0, m1, prm, sd, out=(r0, r1)), steps, warmup),
            "finish_p0": _event_ms(torch, lambda: B.drelu_finish(0, r0, prm, sd, out=y0), steps, warmup),
            "finish_p1": _event_ms(torch, lambda: B.drelu_finish(1, r1, prm, sd, out=y1), steps, warmup),
            "fused": _event_ms(torch, lambda: B.drelu(x0, x1, prm, sd), steps, warmup),
        }
        byt = {"send_p0": 8 + 4 * words, "send_p1": 8 + 4 * words, "reply_p2": 8 * words + 16, "finish_p0": 16,
               "finish_p1": 16}
        r = {k: round(v, 4) for k, v in ms.items()}
        r["parties_sum_ms"] = round(sum(v for k, v in ms.items() if k != "fused"), 4)
        r["message_bytes_per_elem"] = 4 * words
        r["message_bits_theoretical"] = prm.npos * prm.npos
        r["gbs"] = {k: round(b * n / ms[k] / 1e6, 1) for k, b in byt.items()}
        out[name] = r
    return out


def run_streaming(torch, B, inputs, steps, warmup):
    """The HBM-bound streaming calls alone on the 2^24 products z (Z_2^64):
    deterministic truncation (Alg. 5, 13 low bits), SecureML truncation
    (Alg. 1, 13 bits) and the modulo switch (Alg. 6) of the shares read in
    Z_2^60 into Z_p, p = 2^61 - 1.  Algorithmic bytes: both shares in, both
    out, 8 bytes each."""
    z0, z1 = to_dev(torch, inputs[2]), to_dev(torch, inputs[3])
    n = z0.numel()
    out = {"workload": f"{n} shared products in Z_2^64"}
    o0, o1 = torch.empty_like(z0), torch.empty_like(z1)
    calls = (("trunc_det", lambda: B.trunc_det(z0, z1, 64, 13, 0, out=(o0, o1))),
             ("trunc_prob", lambda: B.trunc_prob(z0, z1, 64, 13, out=(o0, o1))))
    for name, fn in calls:
        ms = _event_ms(torch, fn, steps, warmup)
        out[name] = {"ms": round(ms, 4), "gbs": round(32 * n / ms / 1e6, 1),
                     "hbm_frac": round(32 * n / ms / 1e6 / HBM_PEAK_GBS, 4)}
    p = (1 << 61) - 1
    ms = _event_ms(torch, lambda: B.mod_switch(z0, z1, 60, p, out=(o0, o1)), steps, warmup)
    out["mod_switch"] = {"ms": round(ms, 4), "gbs": round(32 * n / ms / 1e6, 1),
                         "hbm_frac": round(32 * n / ms / 1e6 / HBM_PEAK_GBS, 4),
                         "setting": "l' = 60 (shares read mod 2^60), p = 2^61 - 1"}
    return out


def run_copy(torch, steps, warmup, mib=512):
    """A plain device-to-device copy of known size: the reference for achievable
    HBM bandwidth and for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE counters."""
    n = (mib << 20) // 8
    src = torch.empty(n, dtype=torch.int64, device="cuda").fill_(3)
    dst = torch.empty_like(src)
    ms = _event_ms(torch, lambda: dst.copy_(src), steps, warmup)
    return {"bytes_per_copy": 2 * n * 8, "ms": round(ms, 4), "gbs": round(2 * n * 8 / ms / 1e6, 1),
            "hbm_frac": round(2 * n * 8 / ms / 1e6 / HBM_PEAK_GBS, 4)}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sections",
                    default="cpu,alone,streaming,batched,chain,precomputed,rss,linear,split,plain,serving,copy,"
                            "matmul,sweep",
                    help="comma list of extra sections: cpu, alone, streaming, batched, chain, precomputed, rss, "
                         "linear, split, plain, serving, copy, matmul, sweep")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: every step is one GPU's share of the work "
              "(the three parties are simulated on that GPU); --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    sections = {s for s in args.sections.split(",") if s}

    c = KEYBIT
    _, (x0, x1), _, (z0, z1) = W.keybit_drelu(seed=c["seed"], n=c["n"])
    inputs = (x0, x1, z0, z1)

    out = {}
    if "cpu" in sections:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(inputs, min(args.cpu_sample, c["n"]), max(1, args.cpu_workers))
        progress(f"cpu baseline done in {time.perf_counter() - t0:.1f} s")

    import torch
    from paper_2309_04909_amd import bicop as B
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))

    wall, kern = run_keybit(torch, B, inputs, args.steps, args.warmup)
    ms_step = wall / args.steps * 1e3
    value = c["n"] / (ms_step * 1e-3) / 1e9

    ops = alg_ops_per_elem("drelu", c["lx"])
    achieved = ops * c["n"] / (kern["drelu"] * 1e-3) / 1e12
    hbm_bytes = 32 * c["n"]
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": measured_traffic("drelu_keybit"),
                "kernel": "k_drelu<u64, N=19, FieldMersenne<19>>", "ops_per_elem": ops,
                "hbm_alg_bytes_per_launch": hbm_bytes,
                "hbm_frac": round(hbm_bytes / (kern["drelu"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    td_gbs = 32 * c["n"] / (kern["trunc_det"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "warmup_s": round(kern["warmup_s"], 3), "warmup_steps_run": kern["warmup_steps_run"],
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "keybit_drelu: trunc_det(13) of 2^24 products + key-bit DReLU of 2^24 values",
                   "elements": c["n"], "ell": c["ell"], "lx": c["lx"], "k_lo": c["k_lo"], "p": (1 << 19) - 1,
                   "f": 13, "parallelism": "1 GPU, 3 simulated parties",
                   "streams": f"trunc_det on a second stream, {SIDE_TRUNC_BPC} block(s) per CU, beside the DReLU"},
        "roofline": roofline,
        "messages": {"per_element_bits": B.msg_account(B.BC_OP_DRELU, B.Params(c["ell"], c["lx"], c["k_lo"]), 1)["bits"],
                     "rounds": 2, "counted_by": "bc_msg_account (Tab. 1: (l_x + 1)^2 bits per share-holder)"},
        "kernels": {"drelu_ms": round(kern["drelu"], 4), "trunc_det_ms": round(kern["trunc_det"], 4),
                    "drelu_gelem_s": round(c["n"] / kern["drelu"] / 1e6, 3),
                    "trunc_det_in_step_gbs": round(td_gbs, 1), "events": kern["events"], "joins": kern["joins"],
                    "note": "HIP events around each kernel inside the timed steps; the truncation runs on the "
                            "narrow side grid, overlapped with the DReLU (kernels_alone: each on its own)"},
    }
    progress(f"headline: {value:.3f} Gelem/s, {ms_step:.4f} ms per step")
    runs = [("alone", "kernels_alone", lambda: run_alone(torch, B, inputs, 20, 5)),
            ("streaming", "streaming", lambda: run_streaming(torch, B, inputs, 20, 5)),
            ("batched", "batched_vs_plain", lambda: run_batched_vs_plain(torch, B, max(3, args.steps // 5), 2)),
            ("chain", "layer_chain", lambda: run_chain(torch, B, 10, 2)),
            ("precomputed", "precomputed_randomness", lambda: run_precomputed(torch, B, inputs, 10, 2)),
            ("rss", "replicated_sharing", lambda: run_rss(torch, B, inputs, 20, 5)),
            ("linear", "truncate_then_multiply", lambda: run_linear(torch, B, 20, 5)),
            ("split", "parties_apart", lambda: run_split(torch, B, inputs, 20, 5)),
            ("plain", "plain_drelu", lambda: run_plain_drelu(torch, B, args.steps, args.warmup)),
            ("serving", "serving", lambda: run_serving(torch, B)),
            ("matmul", "matmul_relu", lambda: run_matmul_relu(torch, B, args.steps, args.warmup)),
            ("sweep", "batch_sweep", lambda: run_sweep(torch, B, args.steps, args.warmup)),
            ("copy", "copy_reference", lambda: run_copy(torch, args.steps, args.warmup))]
    for sec, key, fn in runs:
        if sec in sections:
            t0 = time.perf_counter()
            line[key] = fn()
            progress(f"section {sec} done in {time.perf_counter() - t0:.1f} s")
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
