"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU.

csrc/api.hip (argument validation, Miller-Rabin and the default primes,
key-bit windows, message accounting, record sizes, ragged-batch plans, the
schedule table) is compiled with both sanitizers on its host side only
(-Xarch_host before each -fsanitize), linked with a driver
(host_sanitize_driver.cpp) that walks every host-only path and every argument
check of the compute calls, and run.  The kernel launchers are replaced by
stubs that return an error: no kernel can run here, and none is needed to
reach the host code.  Any sanitizer report fails the test."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_04909_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _stubs():
    """Definitions of every kernel launcher internal.h declares, each
    returning hipErrorNoDevice."""
    src = open(os.path.join(CSRC, "internal.h")).read()
    out = ['#include "internal.h"', "namespace bc {"]
    for m in re.finditer(r"^hipError_t\s+(\w+)\(([^;]*?)\);", src, flags=re.M | re.S):
        out.append(f"hipError_t {m.group(1)}({m.group(2)}) {{ return hipErrorNoDevice; }}")
    out.append("}  // namespace bc")
    return "\n".join(out) + "\n", len(out) - 3


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and clang++")
def test_host_code_under_asan_and_ubsan(tmp_path):
    stub_src, nstubs = _stubs()
    assert nstubs >= 20
    (tmp_path / "stubs.hip").write_text(stub_src)
    common = ["-O1", "-g", "-std=c++17", "-fPIC", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}"]
    host_only = ["--cuda-host-only", "-x", "hip", "--offload-arch=gfx950"]
    _run([HIPCC, *host_only, *common, *SAN_HOST, "-c", os.path.join(CSRC, "api.hip"), "-o", str(tmp_path / "api.o")])
    _run([HIPCC, *host_only, *common, "-c", str(tmp_path / "stubs.hip"), "-o", str(tmp_path / "stubs.o")])
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    _run([CLANG, *common, *san, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c",
          os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", str(tmp_path / "driver.o")])
    exe = str(tmp_path / "driver")
    _run([CLANG, *san, str(tmp_path / "driver.o"), str(tmp_path / "api.o"), str(tmp_path / "stubs.o"),
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "driver done" in r.stdout, report
    assert re.search(r"check_params ok \d+ bad \d+", r.stdout)
    # the driver's sum of bc_default_prime(0..40) equals the oracle's primes
    from oracle.params import default_prime
    want = sum(default_prime(lx) for lx in range(1, 33))
    got = int(re.search(r"default_prime_sum (\d+)", r.stdout).group(1))
    assert got == want
