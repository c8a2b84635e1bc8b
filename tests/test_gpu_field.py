"""The kernels' Z_p multiply-add (bc_zp_mul_add runs the same field code as
the DReLU/ReLU kernels) against exact integer arithmetic, at the bounds of
every reduction: every window width l_x = 1..32 with its default prime
(fp32 quotient, Mersenne and pseudo-Mersenne folds, 2^33 - 9), and explicit
non-default primes (fp64 quotient, Barrett, 128-bit product).  Operands
cover 0, 1, p - 1, 2^l_x (P0's largest modulo-switch value) and d = p (P1's
p - z when z = 0), plus random triples."""

import numpy as np
import pytest

from oracle.params import default_prime, is_prime

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04909_amd import bicop
    return bicop


def _prev_prime(p):
    c = p - 2
    while not is_prime(c):
        c -= 1
    return c


def _triples(p, lx, rng, k=20000):
    edge_ab = sorted(v for v in {0, 1, 2, p - 1, p - 2, (1 << lx), (1 << lx) - 1, p // 2, p // 3} if 0 <= v < p)
    edge_d = sorted({0, 1, p - 1, p, p // 2})
    a, b, d = [], [], []
    for x in edge_ab:
        for y in edge_ab:
            for z in edge_d:
                a.append(x), b.append(y), d.append(z)
    r = np.random.default_rng(rng)
    ra = [int(v) for v in r.integers(0, p, size=k, dtype=np.uint64)]
    rb = [int(v) for v in r.integers(0, p, size=k, dtype=np.uint64)]
    rd = [int(v) for v in r.integers(0, p + 1, size=k, dtype=np.uint64)]
    return a + ra, b + rb, d + rd


def _run(B, lx, p):
    a, b, d = _triples(p, lx, lx * 7919 + p % 1000)
    t = lambda v: torch.tensor(np.array(v, dtype=np.uint64).view(np.int64), device="cuda")  # noqa: E731
    out = B.zp_mul_add(t(a), t(b), t(d), lx, p)
    got = out.cpu().numpy().view(np.uint64)
    want = np.array([(x * y + z) % p for x, y, z in zip(a, b, d)], dtype=np.uint64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (lx, p, [(a[i], b[i], d[i], int(got[i]), int(want[i])) for i in bad[:3]])


@pytest.mark.parametrize("lx", list(range(1, 33)))
def test_default_prime_fields(B, lx):
    _run(B, lx, default_prime(lx))


@pytest.mark.parametrize("lx", [3, 7, 11, 13, 16, 18, 21, 24, 28, 31, 32])
def test_explicit_prime_fields(B, lx):
    p = _prev_prime(default_prime(lx))
    assert p > (1 << lx)
    _run(B, lx, p)
