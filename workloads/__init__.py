"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds no step of the DReLU/ReLU method: it only draws plaintext
values with the shapes and distributions of the workloads, encodes them as
fixed-point ring elements and splits them into the 2-of-2 input sharing
[x]_0 = x + R, [x]_1 = -R (the input format of every protocol, Sec. 2.2).
Draws use NumPy's PCG64 generator seeded explicitly, so both the CPU oracle
and the GPU path receive byte-identical inputs.

Workloads (values are round-half-even of v * 2^f):
  plain_drelu   65,536 elements, v ~ U(-64, 64), f = 13, l = 64
  keybit_drelu  2^24 elements, v ~ N(0, 8^2) clipped to |x| < 2^30, f = 13,
                l = 64; plus z = x1 * x2 mod 2^64 of two such tensors for the
                13-bit deterministic truncation
  matmul_relu   Z = A B with A [4096 x 4096], B [4096 x 1024], entries
                round(N(0,1) 2^f); exact (every partial sum < 2^53 in fp64);
                f = 13 in Z_{2^64} or f = 8 in Z_{2^32}
  resnet18      the 17 ReLU activation tensors of a ResNet-18 forward pass at
                batch B, 224 x 224 input, values round(N(0,1) 2^13), l = 64
  serving       Poisson arrivals, sizes log-uniform in [2^10, 2^24]
The paper's own inputs (CIFAR10 / Tiny ImageNet activations of trained
AlexNet / VGG16) are not available; these synthetic tensors stand in for them.
"""

import numpy as np

U64 = np.uint64


def storage_dtype(ell: int):
    """Shares of Z_{2^l} are stored in 4 bytes when l <= 32, else 8 bytes."""
    return np.uint32 if ell <= 32 else np.uint64


def fixed_point(v, f: int) -> np.ndarray:
    """round-half-even(v * 2^f) as int64."""
    return np.rint(np.asarray(v, dtype=np.float64) * float(1 << f)).astype(np.int64)


def encode(xi, ell: int) -> np.ndarray:
    """Signed integers -> canonical elements of Z_{2^l} (uint64)."""
    u = np.ascontiguousarray(np.asarray(xi).astype(np.int64)).view(np.uint64)
    if ell < 64:
        u = u & U64((1 << ell) - 1)
    return u


def share(x, ell: int, rng: np.random.Generator):
    """2-of-2 additive sharing with a uniform mask R in Z_{2^l}.

    Returns (x0, x1) in the storage dtype of the ring."""
    x = np.asarray(x, dtype=U64)
    R = rng.bit_generator.random_raw(x.size).astype(U64).reshape(x.shape)
    if ell < 64:
        m = U64((1 << ell) - 1)
        R &= m
        x0 = (x + R) & m
        x1 = (~R + U64(1)) & m
    else:
        x0 = x + R
        x1 = ~R + U64(1)
    dt = storage_dtype(ell)
    return x0.astype(dt), x1.astype(dt)


def share3(x, ell: int, rng: np.random.Generator):
    """Replicated (2-of-3) sharing: x = x0 + x1 + x2 mod 2^l with x0, x1
    uniform.  Returns (x0, x1, x2) in the storage dtype of the ring."""
    x = np.asarray(x, dtype=U64)
    a = rng.bit_generator.random_raw(x.size).astype(U64).reshape(x.shape)
    b = rng.bit_generator.random_raw(x.size).astype(U64).reshape(x.shape)
    c = x - a - b
    if ell < 64:
        m = U64((1 << ell) - 1)
        a, b, c = a & m, b & m, c & m
    dt = storage_dtype(ell)
    return a.astype(dt), b.astype(dt), c.astype(dt)


def signed_values(x, ell: int) -> np.ndarray:
    """Signed int64 view of canonical ring elements (ell <= 64)."""
    x = np.asarray(x, dtype=U64)
    if ell == 64:
        return x.view(np.int64)
    s = x.astype(np.int64)
    return np.where(s >= (1 << (ell - 1)), s - (1 << ell), s)


# ------------------------------------------------------------------ workloads

F = 13


def plain_drelu(seed: int = 1, n: int = 65536):
    rng = np.random.default_rng(seed)
    x = encode(fixed_point(rng.uniform(-64.0, 64.0, size=n), F), 64)
    return x, share(x, 64, rng)


def keybit_values(rng, n):
    v = rng.normal(0.0, 8.0, size=n)
    xi = fixed_point(v, F)
    lim = (1 << 30) - 1
    return np.clip(xi, -lim, lim)


def keybit_drelu(seed: int = 2, n: int = 1 << 24):
    """x for the key-bit DReLU and the product z = x1 * x2 mod 2^64 for the
    13-bit deterministic truncation, both shared in Z_{2^64}."""
    rng = np.random.default_rng(seed)
    xi = keybit_values(rng, n)
    x = encode(xi, 64)
    sx = share(x, 64, rng)
    p1 = keybit_values(rng, n)
    p2 = keybit_values(rng, n)
    z = p1.view(U64) * p2.view(U64)              # wraps mod 2^64; |z| < 2^60
    sz = share(z, 64, rng)
    return x, sx, z, sz


def matmul_product(seed: int = 3, m: int = 4096, k: int = 4096, ncols: int = 1024, f: int = F):
    """Z = A B exactly, entries of A and B round(N(0,1) 2^f) (int64)."""
    rng = np.random.default_rng(seed)
    A = fixed_point(rng.standard_normal((m, k)), f)
    B = fixed_point(rng.standard_normal((k, ncols)), f)
    Zf = A.astype(np.float64) @ B.astype(np.float64)
    assert np.abs(Zf).max() < 2.0 ** 53
    return Zf.astype(np.int64).ravel()


def matmul_relu(seed: int = 3, ell: int = 64, f: int | None = None, m: int = 4096, k: int = 4096, ncols: int = 1024):
    """Shares (in Z_{2^l}) of the exact fixed-point product, before truncation."""
    if f is None:
        f = F if ell == 64 else 8
    Z = matmul_product(seed, m, k, ncols, f)
    z = encode(Z, ell)
    rng = np.random.default_rng(seed + 1000)
    return z, share(z, ell, rng)


RESNET18_SHAPES = (
    [(64, 112, 112)] +
    [(64, 56, 56)] * 4 +
    [(128, 28, 28)] * 4 +
    [(256, 14, 14)] * 4 +
    [(512, 7, 7)] * 4
)


def linear_factors(seed: int = 5, n: int = 1 << 24, f: int = 26, int_bits: int = 5, ell: int = 64):
    """Two tensors of fixed-point factors for one secure multiplication:
    values uniform over the whole domain of int_bits integer and f fractional
    bits (|x| < 2^(int_bits + f), 31 bits at the defaults, the l = 64 setting
    of Sec. 4), each shared 2-of-2.  Returns ((x, (x0, x1)), (y, (y0, y1)))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        v = rng.integers(-(1 << (int_bits + f)) + 1, 1 << (int_bits + f), size=n)
        x = encode(v, ell)
        out.append((x, share(x, ell, rng)))
    return tuple(out)


def resnet18_sizes(batch: int = 32):
    return [batch * c * h * w for (c, h, w) in RESNET18_SHAPES]


def resnet18_relu(seed: int = 4, batch: int = 32, layers=None, f: int = F):
    """List of (x, (x0, x1)) per ReLU tensor of a ResNet-18 pass, flattened:
    N(0, 1) values with f fractional bits in Z_2^64 (f = 2 F: the layer's
    products before their truncation)."""
    rng = np.random.default_rng(seed)
    out = []
    for i, n in enumerate(resnet18_sizes(batch)):
        if layers is not None and i not in layers:
            continue
        x = encode(fixed_point(rng.standard_normal(n), f), 64)
        out.append((x, share(x, 64, rng)))
    return out


def chain_values(seed: int, n: int, f: int = 2 * F):
    """Inputs of one step of a layer chain: n values N(0, 1) at f = 2 F
    fractional bits in Z_2^64 (a layer's products before their truncation by
    F bits), and their 2-of-2 sharing."""
    rng = np.random.default_rng(seed)
    x = encode(fixed_point(rng.standard_normal(n), f), 64)
    return x, share(x, 64, rng)


def serving_arrivals(seed: int, rate_jobs_per_s: float, count: int,
                     min_log2: int = 10, max_log2: int = 24):
    """Seeded Poisson arrivals: (arrival_time_s, n_elems, op, ell) per job.

    op is 'drelu' or 'relu' with probability 1/2, ell is 32 or 64 with
    probability 1/2, sizes log-uniform in [2^min_log2, 2^max_log2]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_jobs_per_s, size=count)
    times = np.cumsum(gaps)
    sizes = np.floor(2.0 ** rng.uniform(min_log2, max_log2, size=count)).astype(np.int64)
    ops = np.where(rng.random(count) < 0.5, "drelu", "relu")
    ells = np.where(rng.random(count) < 0.5, 32, 64)
    return [(float(t), int(s), str(o), int(e)) for t, s, o, e in zip(times, sizes, ops, ells)]


def serving_values(seed: int, n: int, ell: int):
    """Values of one serving job: as keybit_drelu for l = 64; f = 8,
    v ~ N(0, 8^2) for l = 32."""
    rng = np.random.default_rng(seed)
    if ell == 64:
        x = encode(keybit_values(rng, n), 64)
    else:
        xi = fixed_point(rng.normal(0.0, 8.0, size=n), 8)
        lim = (1 << 15) - 1                      # |v| < 128: inside the guard domain of k_lo = 8, l_x = 8
        x = encode(np.clip(xi, -lim, lim), 32)
    return x, share(x, ell, rng)
