"""Maximum sizes: one call on n = 2^31 + 3 elements (16 GiB per share array,
64 GiB on the device), so every index of the grid-stride loops and of the
randomness counters passes 2^31.  Inputs are drawn on the device; outputs are
checked against the oracle on sampled elements, most of them near the end."""

import numpy as np
import pytest

from oracle import protocols as OPR
from oracle.params import default_prime

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = np.uint64
N_HUGE = (1 << 31) + 3


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < 80 << 30:
        pytest.skip("needs 80 GiB of free device memory")
    from paper_2309_04909_amd import bicop
    return bicop


@pytest.fixture(scope="module")
def shares(B):
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    x0 = torch.randint(-(1 << 63), (1 << 63) - 1, (N_HUGE,), dtype=torch.int64, device="cuda", generator=g)
    x1 = torch.randint(-(1 << 63), (1 << 63) - 1, (N_HUGE,), dtype=torch.int64, device="cuda", generator=g)
    y0, y1 = torch.empty_like(x0), torch.empty_like(x1)
    yield x0, x1, y0, y1
    del x0, x1, y0, y1
    torch.cuda.empty_cache()


def _sample(n):
    rng = np.random.default_rng(7)
    idx = np.concatenate([np.arange(64), np.arange((1 << 31) - 64, (1 << 31) + 64),
                          np.arange(n - 64, n), rng.integers(0, n, size=600)])
    return np.unique(idx[idx < n])


def _host(t, idx):
    return t[torch.from_numpy(idx).cuda()].cpu().numpy().view(U64)


def test_trunc_det_past_2p31(B, shares):
    x0, x1, y0, y1 = shares
    B.trunc_det(x0, x1, 64, 13, out=(y0, y1))
    idx = _sample(N_HUGE)
    a0, a1 = _host(x0, idx), _host(x1, idx)
    e0, e1 = OPR.trunc_det(a0, a1, 64, 13)
    assert np.array_equal(_host(y0, idx), e0) and np.array_equal(_host(y1, idx), e1)


@pytest.mark.parametrize("op", ["drelu", "relu"])
def test_drelu_relu_past_2p31(B, shares, op):
    x0, x1, y0, y1 = shares
    prm, seeds, nonce = B.Params(64, 18, 13), (5, 6, 7), 8
    fn, ofn = (B.drelu, OPR.drelu) if op == "drelu" else (B.relu, OPR.relu)
    fn(x0, x1, prm, B.Seeds(*seeds, nonce), out=(y0, y1))
    idx = _sample(N_HUGE)
    o0, o1, _, _ = ofn(_host(x0, idx), _host(x1, idx), 64, 18, 13, default_prime(18), seeds, nonce,
                       g=idx.astype(U64))
    assert np.array_equal(_host(y0, idx), o0) and np.array_equal(_host(y1, idx), o1)
