"""Arithmetic in Z_{2^l} on NumPy uint64 arrays (test infrastructure only).

Canonical representatives lie in [0, 2^l).  The cut function of Sec. 2.3
(drop the low k bits, and optionally the high k2 bits) is a right shift
followed by a reduction; see ``cut``.
"""

import numpy as np

U64 = np.uint64


def as_u64(a):
    return np.asarray(a, dtype=U64)


def mask(bits: int) -> int:
    """2^bits - 1 as a Python int (bits in [0, 64])."""
    return (1 << bits) - 1


def red(a, bits: int):
    """a mod 2^bits for a uint64 array (bits <= 64)."""
    a = as_u64(a)
    if bits >= 64:
        return a.copy()
    return a & U64(mask(bits))


def neg(a, bits: int):
    """-a mod 2^bits."""
    a = as_u64(a)
    return red((~a) + U64(1), bits)


def add(a, b, bits: int):
    return red(as_u64(a) + as_u64(b), bits)


def sub(a, b, bits: int):
    return red(as_u64(a) - as_u64(b), bits)


def mul(a, b, bits: int):
    """a*b mod 2^bits; uint64 multiplication wraps mod 2^64 and 2^bits | 2^64."""
    return red(as_u64(a) * as_u64(b), bits)


def cut(a, k1: int, k2: int, bits: int):
    """cut(a, k1, k2) of Sec. 2.3: the bits [k1, bits-k2) of a, as an integer.

    With k2 = 0 this is cut(a, k) = a >> k.  (The paper's sum writes the
    exponent as 2^i; the binary form it gives shows the intended right shift.)
    """
    assert 0 <= k1 and 0 <= k2 and k1 + k2 <= bits
    a = red(a, bits)
    return red(a >> U64(k1), bits - k1 - k2)


def signed(a, bits: int):
    """Signed value of a canonical element: a - 2^bits * [a >= 2^(bits-1)]
    (Python ints, object array)."""
    a = red(a, bits)
    out = a.astype(object)
    half = 1 << (bits - 1)
    return np.where(a >= U64(half), out - (1 << bits), out)


def from_signed(v, bits: int):
    """Canonical element of Z_{2^bits} for Python-int / int64 values."""
    v = np.asarray(v, dtype=object)
    m = 1 << bits
    return np.array([int(x) % m for x in v.ravel()], dtype=U64).reshape(v.shape)


def split(x, R, bits: int):
    """The 2-of-2 sharing of Sec. 2.2: [x]_0 = x + R, [x]_1 = -R (mod 2^bits)."""
    return add(x, R, bits), neg(R, bits)


def reconstruct(a0, a1, bits: int):
    return add(a0, a1, bits)
