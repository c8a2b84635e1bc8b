"""Build libbicop.so (the C ABI of include/bicop.h) for gfx950 with hipcc.

Every .hip file under csrc/ is compiled to an object in _build/ (in parallel),
then the objects are linked into paper_2309_04909_amd/libbicop.so.  The
packed-fp32 target feature is switched off for all device code.

    python -m paper_2309_04909_amd.build [-j N] [--asm]
"""

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbicop.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-command-line-argument",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # let '#pragma unroll' fully unroll the 33-slot loops of l_x = 32 (else
    # the slot arrays are indexed dynamically, through scratch)
    "-mllvm", "-pragma-unroll-threshold=200000",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return r.returncode, out


def build(jobs: int | None = None, verbose: bool = False, asm: bool = False, extra_flags=(), out: str = LIB,
          build_dir: str = BUILD) -> str:
    """Compile every HIP source and link libbicop.so (or `out`).  Returns the library path."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 4)))

    def compile_one(src):
        obj = os.path.join(build_dir, os.path.basename(src).replace(".hip", ".o"))
        rc, log = _run([HIPCC, *FLAGS, *extra_flags, "-c", src, "-o", obj])
        if rc == 0 and asm:
            s = os.path.join(build_dir, os.path.basename(src).replace(".hip", ".s"))
            _run([HIPCC, *FLAGS, *extra_flags, "--cuda-device-only", "-S", src, "-o", s])
        return src, obj, rc, log

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, srcs))
    errors = [(s, o) for s, _, rc, o in results if rc != 0]
    for s, _, rc, log in results:
        if log and (verbose or rc != 0):
            print(f"--- {os.path.basename(s)}\n{log}", file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed for: " + ", ".join(os.path.basename(s) for s, _ in errors))
    tmp = out + ".tmp"
    rc, log = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[o for _, o, _, _ in results]])
    if rc != 0:
        raise RuntimeError("link failed:\n" + log)
    os.replace(tmp, out)
    return out


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--asm", action="store_true", help="also write device assembly next to the objects")
    a = ap.parse_args()
    print(build(a.j, a.v, a.asm))
