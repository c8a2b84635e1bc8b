"""Protocol parameters (test infrastructure only).

* The prime p of the modulo switch has bit length l_x + 1 (notation table;
  Alg. 6).  The paper names no particular prime; the reading used here is the
  largest prime below 2^(l_x+1), which lies in (2^l_x, 2^(l_x+1)).
* The DReLU windows are trc(x, i, l - l_x - i) for i = 0..l_x (Alg. 7);
  with key bits (Sec. 6.1) the window moves up by k_lo bits, so window i
  drops k_lo + i low bits.  Window i = l_x must fit in the ring:
  k_lo + 2*l_x <= l.
"""

from . import ring  # noqa: F401  (kept for a uniform import surface)

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; exact for n < 3.3e24 with these bases."""
    if n < 2:
        return False
    for q in _MR_BASES:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def default_prime(lx: int) -> int:
    """Largest prime p < 2^(lx+1); it satisfies 2^lx < p (Bertrand)."""
    c = (1 << (lx + 1)) - 1
    while not is_prime(c):
        c -= 1
    assert c > (1 << lx)
    return c


def check_drelu(ell: int, lx: int, k_lo: int, p: int) -> None:
    """Raise ValueError unless (ell, lx, k_lo, p) is a valid DReLU setting."""
    if not (2 <= ell <= 64):
        raise ValueError("ring bit length must be in [2, 64]")
    if lx < 1 or k_lo < 0 or k_lo + 2 * lx > ell:
        raise ValueError("window must satisfy lx >= 1 and k_lo + 2*lx <= ell")
    if lx + 1 > 64:
        raise ValueError("lx too large")
    if not ((1 << lx) < p < (1 << (lx + 1)) and is_prime(p)):
        raise ValueError("p must be a prime in (2^lx, 2^(lx+1))")


def keybit_window(f: int, lx_int: int, lx_frac: int):
    """Key-bit window of Sec. 6.1 for fixed point with f fractional bits.

    The DReLU keeps lx_int integer bits and lx_frac fractional bits of x,
    so it drops the low k_lo = f - lx_frac bits and looks at l_x = lx_int +
    lx_frac bits above them.  Returns (k_lo, l_x).
    """
    if not (0 <= lx_frac <= f):
        raise ValueError("lx_frac must be in [0, f]")
    return f - lx_frac, lx_int + lx_frac


def guard_bound(k_lo: int, lx: int) -> int:
    """Inputs with |x| < 2^(k_lo + lx - 1) leave one guard bit at the top of
    the window; on that domain the sign test is exact outside |x| < 2^k_lo."""
    return 1 << (k_lo + lx - 1)
