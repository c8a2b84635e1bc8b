#!/usr/bin/env python3
"""Benchmark of the Bicoptor 2.0 DReLU/ReLU hot path on one MI355X.

One step is one pass of the key-bit workload: the 13-bit deterministic
truncation (Alg. 5) of 2^24 shared products z = x1 * x2 in Z_{2^64}, followed
by the key-bit DReLU (Alg. 7, l = 64, k_lo = 13, l_x = 18, p = 2^19 - 1) of
2^24 shared fixed-point values x (f = 13, |x| < 2^30).  Inputs are seeded
synthetic data, resident in HBM before timing starts.  `value` is DReLU
elements per second of the whole step.

Printed as one JSON line (rank 0), with extra sections:
  kernels           per-kernel average durations (HIP events on the launch stream)
  roofline          the dominant kernel (the fused DReLU) against its ALU roofline
  cpu_baseline      the CPU oracle timed on a bounded sample of the same workload
  batched_vs_plain  ResNet-18 ragged ReLU: one persistent graph launch vs 17 launches
  serving           continuous-batching request loop: p50/p99 latency and Gelem/s
  plain_drelu       l = 64 without key bits (l_x = 32), 65,536 elements: us per call

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "DReLU Gelem/s (ℓ=64, key bits), batched vs plain, %HBM peak; p50/p99"
HBM_PEAK_GBS = 8000.0
# 32-bit vector ALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz (the rate at
# which simple 32-bit VALU instructions issue; fp32 vector 157.3 TFLOP/s counts
# an FMA as two flops).  VOP3-class instructions (64-bit shifts, 32x32->64
# multiplies, three-operand forms) issue at half this rate.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12

KEYBIT = dict(ell=64, lx=18, k_lo=13, trunc_k=13, n=1 << 24, seed=2)
SEEDS = (0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0)


# ------------------------------------------------------------- ALU op model


def batcher_comparators(n: int) -> int:
    """Comparators of the pruned Batcher network the kernel sorts keys with."""
    P = 1
    while P < n:
        P *= 2
    c = 0
    p = 1
    while p < P:
        k = p
        while k >= 1:
            for j in range(k % p, P - k, 2 * k):
                for i in range(min(k, P - j - k)):
                    if (i + j) // (2 * p) == (i + j + k) // (2 * p) and i + j + k < n:
                        c += 1
            k //= 2
        p *= 2
    return c


PHILOX_OPS = 60          # 10 rounds x (two 32x32->64 multiplies + four XORs)
SLOT_OPS = 40            # per slot: two windows, adjacent sums, mod switch, two draws,
                         # two masked products with reshare, P2's sum and zero test
SLOT_OPS_WIDE = 64       # same with 64-bit field elements (l_x = 32)
TAIL_OPS = {"drelu": 12, "relu": 40}


def alg_ops_per_elem(op: str, lx: int) -> int:
    """32-bit integer operations per element of the fused kernel (the model in the design doc)."""
    n = lx + 1
    wide = lx == 32
    blocks = (n + 3) // 4 + (n if wide else (n + 1) // 2) + (1 if op == "drelu" else 3)
    return (blocks * PHILOX_OPS + n * (SLOT_OPS_WIDE if wide else SLOT_OPS) + 2 * batcher_comparators(n)
            + TAIL_OPS[op])


def source_hash(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2309_04909_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


DRELU_SOURCES = ["bc_device.h", "drelu_kernel.h"]


def measured_traffic(kernel: str, src_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None if the
    kernel sources changed since the counters were taken."""
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
    return {"value": done / dt / 1e9, "unit": "Gelem/s", "cores": workers, "kind": "oracle",
            "sample": f"first {done} elements of the step (13-bit trunc_det of z and key-bit DReLU of x), "
                      f"{workers} processes, {dt:.1f} s wall"}


# ------------------------------------------------------------------- GPU parts


class Timer:
    """HIP events on the stream the kernels are launched on (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def stop(self, name, s):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs.setdefault(name, []).append((s, e))

    def avg_ms(self, name):
        ps = self.pairs.get(name, [])
        return sum(s.elapsed_time(e) for s, e in ps) / max(1, len(ps))


def to_dev(torch, a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()


def run_keybit(torch, B, inputs, steps, warmup):
    c = KEYBIT
    x0, x1, z0, z1 = (to_dev(torch, a) for a in inputs)
    prm = B.Params(c["ell"], c["lx"], c["k_lo"])
    sd = B.Seeds(*SEEDS, 7)
    y0, y1 = torch.empty_like(x0), torch.empty_like(x1)
    t0, t1 = torch.empty_like(z0), torch.empty_like(z1)

    def step(timer=None):
        s = timer.start() if timer else None
        B.trunc_det(z0, z1, c["ell"], c["trunc_k"], 0, out=(t0, t1))
        if timer:
            timer.stop("trunc_det", s)
            s = timer.start()
        B.drelu(x0, x1, prm, sd, out=(y0, y1))
        if timer:
            timer.stop("drelu", s)

    for _ in range(warmup):
        step()
    # the timed region: barrier (single GPU: none) + synchronize on both sides;
    # HIP events between the kernels give their durations
    timer = Timer(torch)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        step(timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    return wall, {"trunc_det": timer.avg_ms("trunc_det"), "drelu": timer.avg_ms("drelu")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sections", default="cpu", help="comma list of extra sections: cpu")
    ap.add_argument("--cpu-sample", type=int, default=1 << 21)
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
        out["cpu_baseline"] = cpu_baseline(inputs, min(args.cpu_sample, c["n"]), max(1, args.cpu_workers))

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
                "traffic": measured_traffic("drelu_keybit", source_hash(DRELU_SOURCES)),
                "kernel": "k_drelu<u64, N=19, FieldMersenne<19>>", "ops_per_elem": ops,
                "hbm_alg_bytes_per_launch": hbm_bytes,
                "hbm_frac": round(hbm_bytes / (kern["drelu"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    td_gbs = 32 * c["n"] / (kern["trunc_det"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "keybit_drelu: trunc_det(13) of 2^24 products + key-bit DReLU of 2^24 values",
                   "elements": c["n"], "ell": c["ell"], "lx": c["lx"], "k_lo": c["k_lo"], "p": (1 << 19) - 1,
                   "f": 13, "parallelism": "1 GPU, 3 simulated parties"},
        "roofline": roofline,
        "kernels": {"drelu_ms": round(kern["drelu"], 4), "trunc_det_ms": round(kern["trunc_det"], 4),
                    "drelu_gelem_s": round(c["n"] / kern["drelu"] / 1e6, 3),
                    "trunc_det_gbs": round(td_gbs, 1), "trunc_det_hbm_frac": round(td_gbs / HBM_PEAK_GBS, 4)},
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
