"""bench.py's host side without a GPU: it refuses more than one GPU with a
message, and its cpu_baseline leg (the oracle on a bounded sample of the
headline step's inputs) reports the fields of the bench line's cpu_baseline
object."""

import importlib.util
import os
import subprocess
import sys

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod          # the forked oracle workers find their function by module name
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_cpu_baseline_fields():
    bench = _bench()
    _, (x0, x1), _, (z0, z1) = W.keybit_drelu(seed=2, n=4096)
    cb = bench.cpu_baseline((x0, x1, z0, z1), 4096, 2)
    assert cb["kind"] == "oracle" and cb["unit"] == "Gelem/s" and cb["cores"] == 2
    assert cb["value"] > 0 and cb["single_process"]["elements"] == 4096
    assert cb["sample"].startswith("first 4096 elements")
