"""Autotuner: picks launch schedules on the GPU and writes schedules.json.

For each kernel kind and setting of the workloads it times a sweep of grid
sizes (blocks of 256 threads per compute unit, so elements per thread
= n / (grid * 256)), for the DReLU and the ReLU kernels apart; for small
calls it sweeps the lanes per element (1, 4 or 8 lanes share an element);
for the ragged batch it also sweeps the tile size.  Entries are keyed by
(kind, window count, storage width, op), the key of the library's table, so
two settings that share a window count keep their own schedules.  Results
never depend on the schedule (checked here on every candidate); only speed
does.  The binding applies schedules.json at import.

    python -m paper_2309_04909_amd.tune [--quick]
"""

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import bicop as B

HERE = os.path.dirname(os.path.abspath(__file__))

# (ell, lx, k_lo) of the workloads: key-bit DReLU, ResNet ReLU, matmul ReLU
# (both rings), serving l = 32, plain DReLU (l_x = 31 and 32)
SETTINGS = [(64, 18, 13), (64, 7, 11), (51, 11, 13), (24, 7, 10), (32, 8, 8), (64, 31, 0), (64, 32, 0)]
BPC = [1, 2, 4, 8, 16, 32, 64]
TILES = [256, 512, 1024, 2048, 4096, 8192]


def _time(fn, reps=10, warm=2, rounds=3):
    """Milliseconds per call: the best of `rounds` timings of `reps` calls
    (a single round caught clock ramps and let close candidates swap places
    between tuning runs)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(rounds):
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        best = ms if best is None or ms < best else best
    return best


def _time_graph(fn, reps=20, replays=5):
    """GPU milliseconds per call of fn, with `reps` calls captured into one HIP
    graph and the graph replayed: small calls are not timed by the host's
    launch rate.  fn must enqueue GPU work only (outputs preallocated)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(replays):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (replays * reps)


def _shares(n, ell, seed):
    rng = np.random.default_rng(seed)
    dt = np.uint64 if ell > 32 else np.uint32
    view = torch.int64 if ell > 32 else torch.int32
    x0 = torch.from_numpy(rng.integers(0, 2 ** 62, size=n, dtype=np.int64).astype(dt).view(
        np.int64 if ell > 32 else np.int32)).cuda().view(view)
    x1 = torch.from_numpy(rng.integers(0, 2 ** 62, size=n, dtype=np.int64).astype(dt).view(
        np.int64 if ell > 32 else np.int32)).cuda().view(view)
    return x0, x1


def _same(a, b):
    return torch.equal(a[0].view(torch.int64 if a[0].element_size() == 8 else torch.int32),
                       b[0].view(torch.int64 if b[0].element_size() == 8 else torch.int32)) and \
        torch.equal(a[1].view(torch.int64 if a[1].element_size() == 8 else torch.int32),
                    b[1].view(torch.int64 if b[1].element_size() == 8 else torch.int32))


def tune_kind(kind, settings, n, reps, ops=(B.BC_OP_DRELU, B.BC_OP_RELU)):
    """Grid sweep of the fused ("fused"), online ("pre") or offline ("expand")
    kernels, for each setting and op."""
    out = []
    for ell, lx, k_lo in settings:
        prm = B.Params(ell, lx, k_lo)
        npos, width = lx + 1, B.ring_width(ell)
        x0, x1 = _shares(n, ell, ell + lx)
        y0, y1 = torch.empty_like(x0), torch.empty_like(x1)
        sd = B.Seeds(1, 2, 3, 4)
        for op in ops:
            relu = op == B.BC_OP_RELU
            rand = B.rand_expand(op, prm, sd, n) if kind in ("pre", "expand") else None
            if kind == "fused":
                f = B.relu if relu else B.drelu
                fn = lambda: f(x0, x1, prm, sd, out=(y0, y1))  # noqa: E731
            elif kind == "pre":
                f = B.relu_pre if relu else B.drelu_pre
                fn = lambda: f(x0, x1, prm, rand, out=(y0, y1))  # noqa: E731
            else:
                fn = lambda: B.rand_expand(op, prm, sd, n, out=rand)  # noqa: E731
            ref, best = None, None
            for bpc in BPC:
                B.set_schedule(kind, npos, bpc, width, op)
                ms = _time(fn, reps)
                if kind != "expand":
                    got = (y0.clone(), y1.clone())
                    ref = ref or got
                    assert _same(ref, got), "schedule changed a result"
                if best is None or ms < best[1]:
                    best = (bpc, ms)
                print(f"  {kind:6s} op={op} l={ell} lx={lx:2d} bpc={bpc:3d}: {ms:.3f} ms", flush=True)
            B.set_schedule(kind, npos, best[0], width, op)
            out.append({"kind": kind, "npos": npos, "width": width, "op": op, "blocks_per_cu": best[0],
                        "ms": round(best[1], 4), "n": n, "setting": [ell, lx, k_lo]})
    return out


def tune_group(settings, reps, sizes=(1024, 4096, 16384)):
    """Lanes per element of small calls: the largest group (1, 4 or 8 lanes)
    the library may use, chosen by the summed time over small call sizes."""
    out = []
    for ell, lx, k_lo in settings:
        prm = B.Params(ell, lx, k_lo)
        npos, width = lx + 1, B.ring_width(ell)
        sd = B.Seeds(1, 2, 3, 4)
        calls = [_shares(n, ell, n + lx) for n in sizes]
        outs_buf = [(torch.empty_like(x0), torch.empty_like(x1)) for x0, x1 in calls]
        for op in (B.BC_OP_DRELU, B.BC_OP_RELU):
            f = B.relu if op == B.BC_OP_RELU else B.drelu
            best, ref = None, None
            B.set_schedule("group_fill", npos, 1, width, op)     # groups within one wave per SIMD here
            for gmax in (1, 4, 8):
                B.set_schedule("group", npos, gmax, width, op)
                total, outs = 0.0, []
                for (x0, x1), o in zip(calls, outs_buf):
                    total += _time_graph(lambda: f(x0, x1, prm, sd, out=o), reps * 2)
                    outs.append(f(x0, x1, prm, sd))
                ref = ref or outs
                assert all(_same(a, b) for a, b in zip(ref, outs)), "lanes per element changed a result"
                print(f"  group  op={op} l={ell} lx={lx:2d} lanes<={gmax}: {total * 1e3:.1f} us", flush=True)
                if best is None or total < best[1]:
                    best = (gmax, total)
            B.set_schedule("group", npos, best[0], width, op)
            out.append({"kind": "group", "npos": npos, "width": width, "op": op, "blocks_per_cu": best[0],
                        "ms": round(best[1], 4), "sizes": list(sizes), "setting": [ell, lx, k_lo]})
    return out


def tune_group_fill(settings, reps, sizes=(16384, 32768, 65536)):
    """How many waves per SIMD lane groups may fill (1, 2 or 4): at the
    larger call sizes one lane per element leaves each SIMD with one or two
    long dependent chains, while lane groups split the slots over more waves
    and repeat the shuffle in each.  Chosen by the summed time over sizes,
    with the group schedule already set."""
    out = []
    for ell, lx, k_lo in settings:
        prm = B.Params(ell, lx, k_lo)
        npos, width = lx + 1, B.ring_width(ell)
        sd = B.Seeds(1, 2, 3, 4)
        calls = [_shares(n, ell, n + lx + 1) for n in sizes]
        outs_buf = [(torch.empty_like(x0), torch.empty_like(x1)) for x0, x1 in calls]
        for op in (B.BC_OP_DRELU, B.BC_OP_RELU):
            f = B.relu if op == B.BC_OP_RELU else B.drelu
            best, ref = None, None
            for fill in (1, 2, 4):
                B.set_schedule("group_fill", npos, fill, width, op)
                total, outs = 0.0, []
                for (x0, x1), o in zip(calls, outs_buf):
                    total += _time_graph(lambda: f(x0, x1, prm, sd, out=o), reps * 2)
                    outs.append(f(x0, x1, prm, sd))
                ref = ref or outs
                assert all(_same(a, b) for a, b in zip(ref, outs)), "lane groups changed a result"
                print(f"  fill   op={op} l={ell} lx={lx:2d} waves<={fill}: {total * 1e3:.1f} us", flush=True)
                if best is None or total < best[1]:
                    best = (fill, total)
            B.set_schedule("group_fill", npos, best[0], width, op)
            out.append({"kind": "group_fill", "npos": npos, "width": width, "op": op, "blocks_per_cu": best[0],
                        "ms": round(best[1], 4), "sizes": list(sizes), "setting": [ell, lx, k_lo]})
    return out


def tune_stream(n, reps):
    x0, x1 = _shares(n, 64, 9)
    y0, y1 = torch.empty_like(x0), torch.empty_like(x1)
    best = None
    for bpc in BPC:
        B.set_schedule("stream", 0, bpc, 8)
        ms = _time(lambda: B.trunc_det(x0, x1, 64, 13, out=(y0, y1)), reps)
        print(f"  stream bpc={bpc:3d}: {ms:.4f} ms ({32 * n / ms / 1e6:.0f} GB/s)", flush=True)
        if best is None or ms < best[1]:
            best = (bpc, ms)
    B.set_schedule("stream", 0, best[0], 8)
    return [{"kind": "stream", "npos": 0, "width": 8, "op": 0, "blocks_per_cu": best[0], "ms": round(best[1], 4),
             "n": n}]


def tune_batch(reps, batches=(1, 32)):
    """ResNet-18-shaped ragged batch (l = 64, l_x = 7): tile size x grid,
    timed at each batch size and chosen by the summed time relative to each
    size's best (large tiles suit batch 32 and starve batch 1)."""
    from . import batch as BT
    import workloads as W
    prm = B.Params(64, 7, 11)
    times = {}
    for batch in batches:
        segs = []
        for i, n in enumerate(W.resnet18_sizes(batch)):
            x0, x1 = _shares(n, 64, 100 + i)
            segs.append(BT.Segment(x0, x1, torch.empty_like(x0), torch.empty_like(x1), op=B.BC_OP_RELU, nonce=i))
        for tile in TILES:
            for bpc in (4, 8, 16, 32, 64, 128):
                B.set_schedule("batch", 8, bpc, 8, 0)
                rb = BT.RaggedBatch(prm, B.Seeds(1, 2, 3), segs, tile_elems=tile)
                ms = _time(rb.run, reps)
                times[(batch, tile, bpc)] = ms
                print(f"  batch {batch:2d} tile={tile:5d} bpc={bpc:3d}: {ms:.3f} ms", flush=True)
        del segs
    low = {b: min(v for (bb, _, _), v in times.items() if bb == b) for b in batches}
    score = {}
    for (b, tile, bpc), ms in times.items():
        score[(tile, bpc)] = score.get((tile, bpc), 0.0) + ms / low[b]
    tile, bpc = min(score, key=score.get)
    B.set_schedule("batch", 8, bpc, 8, 0)
    ms = times[(max(batches), tile, bpc)]
    return [{"kind": "batch", "npos": 8, "width": 8, "op": 0, "blocks_per_cu": bpc, "ms": round(ms, 4),
             "batches": list(batches)}], tile


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=B.SCHEDULES_PATH)
    a = ap.parse_args()
    if not torch.cuda.is_available():
        print("the autotuner needs a GPU", file=sys.stderr)
        sys.exit(2)
    n = 1 << (21 if a.quick else 24)              # the size bench.py times
    reps = 5 if a.quick else 10
    t0 = time.time()
    grid = []
    grid += tune_stream(n, reps)
    grid += tune_kind("fused", SETTINGS, n, reps)
    grid += tune_kind("pre", SETTINGS[:5], n, reps)
    grid += tune_kind("expand", SETTINGS[:5], n, reps)
    grid += tune_group(SETTINGS, reps)
    grid += tune_group_fill(SETTINGS, reps)
    bgrid, tile = tune_batch(reps)
    grid += bgrid
    keys = [B.schedule_key(e) for e in grid]
    assert len(keys) == len(set(keys)), "two entries share a key"
    table = {"device": torch.cuda.get_device_name(0), "grid": grid, "batch_tile": tile,
             "tuned_seconds": round(time.time() - t0, 1)}
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table))


if __name__ == "__main__":
    main()
