"""The oracle's Philox4x32-10 against an independent implementation:
rocRAND's header-only engine (ROCm's open-source library), compiled here
for the host by tests/philox_rocrand_ref.cpp.  No GPU.

The engine is keyed by a 64-bit seed (key word 0 = its low half) and runs a
128-bit counter from subsequence * 2^64 + offset / 4, taking the four words
of each block in order; so its output is philox4x32_10 at counter words
(c0, c1) = the low 64 bits and (c2, c3) = the subsequence.  Subsequences with
both halves nonzero reach every counter word, seeds with both halves nonzero
every key word, and an offset that is not a multiple of 4 starts mid-block.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

pytestmark = pytest.mark.skipif(HIPCC is None or not os.path.exists(HEADER),
                                reason="hipcc or rocRAND's headers are not installed")

M32 = (1 << 32) - 1
CASES = [  # (seed, subsequence, offset in words, words)
    (0, 0, 0, 64),
    (0x0123456789ABCDEF, 0, 0, 64),
    (0x0123456789ABCDEF, 0, 4000, 64),
    ((1 << 64) - 1, 0, 4 * ((1 << 32) + 7), 32),          # counter word 1 nonzero
    (0x243F6A8885A308D3, 1, 0, 16),
    (0x243F6A8885A308D3, 0xDEADBEEF12345678, 8, 32),       # counter words 2 and 3 nonzero
    (0x13198A2E03707344, (1 << 64) - 1, 4 * 0xFFFFFFF0, 128),  # word 0 carries into word 1
    (0xA4093822299F31D0, 0x0000000100000000, 6, 30),       # starts at word 2 of block 1
]


@pytest.fixture(scope="module")
def ref(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand_ref")
    subprocess.run([HIPCC, "-O1", os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe], check=True,
                   capture_output=True, timeout=600)
    return exe


def _oracle_words(seed, sub, off, count):
    j = np.arange(off, off + count, dtype=object)
    low = [int(v) // 4 for v in j]                               # the counter's low 64 bits per word
    c0 = np.array([v & M32 for v in low], dtype=np.uint64)
    c1 = np.array([v >> 32 for v in low], dtype=np.uint64)
    c2 = np.full(count, sub & M32, dtype=np.uint64)
    c3 = np.full(count, sub >> 32, dtype=np.uint64)
    w = np.stack(philox4x32_10(c0, c1, c2, c3, seed & M32, seed >> 32), axis=1)
    return w[np.arange(count), np.array([int(v) % 4 for v in j])]


def test_oracle_philox_matches_rocrand_engine(ref):
    text = "".join(f"{s} {u} {o} {c}\n" for s, u, o, c in CASES)
    out = subprocess.run([ref], input=text, capture_output=True, text=True, check=True, timeout=60).stdout.split()
    got = np.array([int(v) for v in out], dtype=np.uint64)
    assert got.size == sum(c for *_, c in CASES)
    pos = 0
    for seed, sub, off, count in CASES:
        exp = _oracle_words(seed, sub, off, count)
        assert np.array_equal(got[pos:pos + count], exp), (hex(seed), hex(sub), off)
        pos += count
