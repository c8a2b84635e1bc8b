"""Summarise rocprofv3 runs of bench.py into profiles/.

Inputs are the output directories of four runs of the same command:
  --trace   rocprofv3 --kernel-trace --stats (with --timed-calls K, the
            mean of each kernel's last K dispatches is listed beside the
            all-call average: the timed steps without the warm-up launches)
  --fetch   rocprofv3 --pmc FETCH_SIZE
  --write   rocprofv3 --pmc WRITE_SIZE
  --valu    rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES SQ_ACTIVE_INST_VALU GRBM_GUI_ACTIVE   (optional)
FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for the plain device copy bench.py runs (copy_reference: a
known number of bytes read and written), giving HBM bytes per launch.

Writes profiles/<name>_kernel_stats.md, profiles/<name>_counters.md and
profiles/traffic.json (bytes per launch per kernel, with the hash of the
kernel sources they were measured on; bench.py reports null for a kernel
whose sources changed since).  Given --trace alone it writes only the
kernel statistics.

    python -m paper_2309_04909_amd.prof_summary --trace D1 --fetch D2 --write D3 [--valu D4] \\
        --name bench_keybit --cmd "<the profiled command>"
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")

# kernel key -> (substring of the demangled name, sources the kernel is built from, algorithmic bytes per launch)
N_KEYBIT = 1 << 24
KERNELS = {
    "drelu_keybit": ("k_drelu<unsigned long, 19, bc::FieldMersenne<19>, false, false>",
                     ["bc_device.h", "drelu_kernel.h"], 32 * N_KEYBIT),
    "trunc_det_keybit": ("OpTruncDet<unsigned long, unsigned long>", ["bc_device.h", "k_stream.hip"],
                         32 * N_KEYBIT),
    # the online kernels of the precomputed mode: shares plus the record (124 B per element at
    # N = 19 for the DReLU, 32 B at N = 8 for the ReLU)
    "drelu_pre_lx18": ("k_drelu_pre<unsigned long, 19, bc::FieldMersenne<19>, false, false>",
                       ["bc_device.h", "drelu_kernel.h", "pre_kernel.h"], (32 + 124) * N_KEYBIT),
    "relu_pre_lx7": ("k_drelu_pre<unsigned long, 8, bc::FieldPM<8, 5u>, true, false>",
                     ["bc_device.h", "drelu_kernel.h", "pre_kernel.h"], (32 + 32) * N_KEYBIT),
}
COPY_BYTES = 512 << 20          # bench.py copy_reference: 512 MiB read and 512 MiB written per copy


_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/', re.S)


def code_text(src: str) -> str:
    """C++ source with comments removed and whitespace runs collapsed, so that
    an edit of comments or layout leaves the hash (and the counters it
    validates) in place."""
    def keep(m):
        t = m.group(0)
        return " " if t.startswith("/") else t
    return " ".join(_TOKENS.sub(keep, src).split())


def source_hash(names, read=None):
    """Hash of the code (not the comments) of csrc/ files; read(name) -> str
    overrides reading the working tree."""
    h = hashlib.sha256()
    for nm in names:
        if read is None:
            with open(os.path.join(HERE, "csrc", nm), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(nm)
        h.update(code_text(text).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _rows(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    out = []
    for fn in files:
        with open(fn, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def kernel_stats(d):
    return [r for r in _rows(d, "kernel_stats.csv")]


def counters(d):
    """{(kernel name, counter): [value per dispatch]}"""
    acc = defaultdict(list)
    for r in _rows(d, "counter_collection.csv"):
        acc[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return acc


XCDS = 8            # MI355X: GRBM_GUI_ACTIVE is reported summed over its 8 accelerator dies
CUS = 256
SIMDS = 4 * CUS


def valu_busy(vc, k):
    """(VALUBusy in %, cycles per VALU wave-instruction per SIMD) of kernel k
    from SQ_ACTIVE_INST_VALU (quad-cycles, summed over SIMDs), SQ_INSTS_VALU
    and GRBM_GUI_ACTIVE (summed over the dies; its per-die value is the
    kernel's cycles).  VALUBusy is rocprofv3's expression
    100 * sum(SQ_ACTIVE_INST_VALU) / CU_NUM / max(GRBM_GUI_ACTIVE)."""
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    if (k, "GRBM_GUI_ACTIVE") not in vc or (k, "SQ_ACTIVE_INST_VALU") not in vc:
        return None, None
    cyc = mean(vc[(k, "GRBM_GUI_ACTIVE")]) / XCDS
    busy = 100 * mean(vc[(k, "SQ_ACTIVE_INST_VALU")]) / CUS / cyc
    per = cyc / (mean(vc[(k, "SQ_INSTS_VALU")]) / SIMDS) if (k, "SQ_INSTS_VALU") in vc else None
    return busy, per


def last_calls_mean(d, k):
    """{kernel name: mean duration in ns of its last k dispatches} from the
    kernel trace (dispatches ordered by start time)."""
    per = defaultdict(list)
    for r in _rows(d, "kernel_trace.csv"):
        per[r["Kernel_Name"]].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = {}
    for name, v in per.items():
        v.sort()
        tail = [dur for _, dur in v[-k:]]
        out[name] = sum(tail) / len(tail)
    return out


def _match(name, key):
    return key in name


def _copy_name(names):
    cands = [n for n in names if "copy" in n.lower()]
    return cands[0] if cands else None


def summarise(trace, fetch, write, valu, name, cmd, timed_calls=0):
    os.makedirs(PROFILES, exist_ok=True)
    stats = kernel_stats(trace)
    last = last_calls_mean(trace, timed_calls) if timed_calls else {}
    extra = f" Last {timed_calls} calls (us) |" if timed_calls else ""
    lines = [f"# rocprofv3 kernel statistics: {name}", "", f"Command: `{cmd}`", "",
             "| Kernel | Calls | Average (us) | Total (ms) | Share |" + extra,
             "|---|---|---|---|---|" + ("---|" if timed_calls else "")]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0))):
        col = ""
        if timed_calls:
            col = f" {last[r['Name']] / 1e3:.2f} |" if r["Name"] in last else " |"
        lines.append(f"| `{r['Name'][:150]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f}% |" + col)
    with open(os.path.join(PROFILES, f"{name}_kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    if fetch is None or write is None:
        return None

    fc, wc = counters(fetch), counters(write)
    names = sorted({k for k, _ in fc} | {k for k, _ in wc})
    copy = _copy_name(names)
    if copy is None:
        raise SystemExit("no copy kernel found in the counter runs")
    mean = lambda v: sum(v) / len(v)  # noqa: E731

    def big(v):
        # the bench's 512 MiB copies: other sections' small copies of the same
        # kernel (plans, records) are left out of the calibration
        return [x for x in v if x >= 0.5 * max(v)]

    scale_f = COPY_BYTES / (mean(big(fc[(copy, "FETCH_SIZE")])) * 1024)
    scale_w = COPY_BYTES / (mean(big(wc[(copy, "WRITE_SIZE")])) * 1024)
    vc = counters(valu) if valu else {}
    tab = ["# HBM traffic and VALU instructions per launch: " + name, "", f"Command: `{cmd}`", "",
           f"Counters scaled by the plain copy `{copy[:80]}` of {COPY_BYTES} B read + {COPY_BYTES} B written: "
           f"FETCH_SIZE x {scale_f:.4f}, WRITE_SIZE x {scale_w:.4f}.", "",
           "| Kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | Algorithmic bytes | Ratio | "
           "VALU instr / wave | VALUBusy | cycles / VALU instr / SIMD |", "|---|---|---|---|---|---|---|---|---|"]
    traffic = {}
    path = os.path.join(PROFILES, "traffic.json")
    if os.path.exists(path):
        with open(path) as f:
            traffic = json.load(f)
    for key, (sub, srcs, alg) in KERNELS.items():
        kn = [n for n in names if _match(n, sub)]
        if not kn:
            continue
        k = kn[0]
        fk, wk = mean(fc[(k, "FETCH_SIZE")]), mean(wc[(k, "WRITE_SIZE")])
        hbm = fk * 1024 * scale_f + wk * 1024 * scale_w
        vi = vb = vp = ""
        if vc:
            vk = [n for n in {a for a, _ in vc} if _match(n, sub)]
            if vk and (vk[0], "SQ_INSTS_VALU") in vc and (vk[0], "SQ_WAVES") in vc:
                vi = f"{mean(vc[(vk[0], 'SQ_INSTS_VALU')]) / mean(vc[(vk[0], 'SQ_WAVES')]):.0f}"
            if vk:
                b, per = valu_busy(vc, vk[0])
                vb = f"{b:.1f}%" if b is not None else ""
                vp = f"{per:.2f}" if per is not None else ""
        tab.append(f"| `{key}` | {fk:.0f} | {wk:.0f} | {hbm:.4g} | {alg:.4g} | {hbm / alg:.3f} | {vi} | {vb} | {vp} |")
        traffic[key] = {"bytes_per_launch": round(hbm), "fetch_kib": fk, "write_kib": wk,
                        "scale_fetch": scale_f, "scale_write": scale_w, "algorithmic_bytes": alg,
                        "source_hash": source_hash(srcs), "command": cmd}
    tab += ["", "VALUBusy is rocprofv3's expression 100 * sum(SQ_ACTIVE_INST_VALU) / CU_NUM / max(GRBM_GUI_ACTIVE), "
            f"with GRBM_GUI_ACTIVE divided by the {XCDS} dies it is summed over (its per-die value over the kernel's "
            "duration gives the ~2.4 GHz counter clock). On gfx950 SQ_ACTIVE_INST_VALU equals SQ_INSTS_VALU: one "
            "quad-cycle per wave instruction, while simple VOP2 operations issue two per quad-cycle, so VALUBusy can "
            "exceed 100%. Cycles per VALU instruction per SIMD = per-die GRBM_GUI_ACTIVE / (SQ_INSTS_VALU / "
            f"{SIMDS} SIMDs): 4 for an issue-bound stream of half-rate (VOP3-class) instructions, about 2 for "
            "full-rate ones."]
    with open(os.path.join(PROFILES, f"{name}_counters.md"), "w") as f:
        f.write("\n".join(tab) + "\n")
    with open(path, "w") as f:
        json.dump(traffic, f, indent=1)
    return traffic


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", default=None, help="without --fetch and --write only the kernel statistics are written")
    ap.add_argument("--write", default=None)
    ap.add_argument("--valu", default=None)
    ap.add_argument("--name", default="bench_keybit")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--timed-calls", type=int, default=0)
    a = ap.parse_args()
    print(json.dumps(summarise(a.trace, a.fetch, a.write, a.valu, a.name, a.cmd, a.timed_calls), indent=1))


if __name__ == "__main__":
    main()
