"""bench.py's ALU op model counts the sorting network the kernels use.

The pruned pairwise network must sort (every 0/1 input up to N = 20, by the
0-1 principle, and random keys above), and its size must be the kernels'
(91 comparators at N = 19, 207 at N = 33, as the device code's constexpr
count gives).  No GPU."""

import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _apply(net, v):
    v = v.copy()
    for lo, hi in net:
        a, b = v[:, lo].copy(), v[:, hi].copy()
        v[:, lo], v[:, hi] = np.minimum(a, b), np.maximum(a, b)
    return v


@pytest.mark.parametrize("n", list(range(2, 21)))
def test_pairwise_network_sorts_every_01_input(bench, n):
    net = bench.pairwise_network(n)
    assert all(0 <= lo < hi < n for lo, hi in net)
    v = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
    out = _apply(net, v)
    assert np.all(out[:, :-1] <= out[:, 1:])


@pytest.mark.parametrize("n", [21, 25, 28, 32, 33])
def test_pairwise_network_sorts_random_keys(bench, n):
    net = bench.pairwise_network(n)
    v = np.random.default_rng(n).integers(0, 1 << 20, size=(20000, n))
    assert np.array_equal(_apply(net, v), np.sort(v, axis=1))


def test_network_sizes_and_op_model(bench):
    sizes = {n: len(bench.pairwise_network(n)) for n in (8, 19, 33)}
    assert sizes == {8: 19, 19: 91, 33: 207}
    # the headline's N = 19 DReLU: 13 Philox blocks (5 for the keys, 7 for the
    # masks at three slots a block, 1 for rho), 19 slots, 91 comparators, the tail
    assert bench.alg_ops_per_elem("drelu", 18) == 13 * 60 + 19 * 40 + 2 * 91 + 12
    # N = 8 (two slots a block) and N = 33 (one): 2 + 4 + 1 and 9 + 33 + 1 blocks
    assert bench.alg_ops_per_elem("drelu", 7) == 7 * 60 + 8 * 40 + 2 * 19 + 12
    assert [bench.mask_blocks(n) for n in (16, 17, 21, 22, 33)] == [8, 6, 7, 11, 33]
