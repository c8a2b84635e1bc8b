"""bench.py's ALU op model: Philox blocks, slots and shuffle digits per
element, with the shuffle's block count from the kernels' chunking rule (the
digits of radices 2, 2, 3, ..., N in 64-bit chunks whose radices multiply to
at most 2^32, two chunks to a block).  No GPU."""

import importlib.util
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("n", range(2, 34))
def test_shuffle_blocks_hold_the_permutation(bench, n):
    blocks = bench.shuffle_blocks(n)
    # the blocks' chunks hold the radices' product 2 n! (at most 2^32 per 64-bit chunk)
    assert 2 * math.factorial(n) <= 1 << (64 * blocks)
    assert blocks == (1 if n <= 19 else 2 if n <= 32 else 3)


def test_op_model(bench):
    # the headline's N = 19 DReLU: 8 Philox blocks (1 for the shuffle, 6 for the
    # 38 mask fields of 19 bits, 1 for rho), 19 slots and 19 digits, the tail
    assert bench.alg_ops_per_elem("drelu", 18) == 8 * 60 + 19 * (40 + 6) + 12
    # N = 8 (two slots a block) and N = 33 (66 fields of 33 bits): 1 + 4 + 1 and 3 + 18 + 1 blocks
    assert bench.alg_ops_per_elem("drelu", 7) == 6 * 60 + 8 * (40 + 6) + 12
    assert bench.alg_ops_per_elem("drelu", 32) == 22 * 60 + 33 * (64 + 6) + 12
    assert [bench.mask_blocks(n) for n in (16, 17, 19, 21, 22, 33)] == [8, 5, 6, 7, 8, 18]
