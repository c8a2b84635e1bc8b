"""Closed forms of the DReLU output and round-1 messages, derived from the
lemmas of the appendix (the patterns of trc over consecutive windows) and
checked by brute force in test_oracle_drelu.py.  Shared by the oracle tests
of the 2-of-2 (Alg. 7, 8) and replicated-sharing (Alg. drelu2) protocols.

x is the secret, Rp the share offset R' = -[x]_1 mod 2^l of the 2-of-2
input (so [x]_0 = x + R'), t the flip bit.
"""

import numpy as np

U = np.uint64


def expected_dprime(x, Rp, t, ell, k_lo):
    """D' of the closed form, per element (Python ints)."""
    out = []
    for xv, rv, tv in zip(x.tolist(), Rp.tolist(), t.tolist()):
        xs = xv - (1 << ell) if xv >> (ell - 1) else xv
        xt = -xs if tv else xs
        Rt = (-rv) % (1 << ell) if tv else rv
        yt = xt >> k_lo
        if yt >= 1:
            out.append(1)
        elif yt <= -1:
            out.append(0)
        else:
            lo = (1 << k_lo) - 1
            out.append(int((xt & lo) + (Rt & lo) >= (1 << k_lo)) if k_lo else 0)
    return np.array(out, dtype=U)


def in_exact_domain(x, t, ell, lx, k_lo):
    res = []
    lo_bound = -((((1 << (lx + 1)) - 2) + 2) // 3)       # -ceil((2^(lx+1)-2)/3)
    for xv, tv in zip(x.tolist(), t.tolist()):
        xs = xv - (1 << ell) if xv >> (ell - 1) else xv
        yt = (-xs if tv else xs) >> k_lo
        hi = (1 << lx) - (1 if k_lo else 0)
        res.append(lo_bound < yt <= hi)
    return np.array(res, dtype=bool)


def expected_zero_count(x, Rp, t, ell, lx, k_lo):
    """Number of i in [0, l_x] with u_i + u_{i+1} - 1 = 0 mod 2^l_x (u_{l_x+1} = 0),
    where u_i = floor(x_t / 2^(k_lo+i)) + e0_i mod 2^l_x (exact e0 of Alg. 5)."""
    out = []
    m = 1 << lx
    for xv, rv, tv in zip(x.tolist(), Rp.tolist(), t.tolist()):
        xs = xv - (1 << ell) if xv >> (ell - 1) else xv
        xt = -xs if tv else xs
        Rt = (-rv) % (1 << ell) if tv else rv
        u = []
        for i in range(lx + 1):
            k = k_lo + i
            lo = (1 << k) - 1
            e0 = int((xt & lo) + (Rt & lo) >= (1 << k)) if k else 0
            u.append(((xt >> k) + e0) % m)
        u.append(0)
        out.append(sum(1 for i in range(lx + 1) if (u[i] + u[i + 1] - 1) % m == 0))
    return np.array(out)


def expected_trunc_prob(x, R, ell, k):
    """Reconstruction of Alg. 1 (SecureML) on x shared as (x + R, -R): the
    exact form floor(sgn(x) / 2^k) + e0 + 2^(l-k) ([x < 0] - [x + R >= 2^l])
    mod 2^l, with e0 = [(x mod 2^k) + (R mod 2^k) >= 2^k] and x, R canonical.
    The last term is e1.  Python ints, per element."""
    out = []
    for xv, rv in zip(x.tolist(), R.tolist()):
        xs = xv - (1 << ell) if xv >> (ell - 1) else xv
        lo = (1 << k) - 1
        e0 = ((xv & lo) + (rv & lo)) >> k
        wrap = (xv + rv) >> ell
        out.append(((xs >> k) + e0 + (1 << (ell - k)) * ((xv >> (ell - 1)) - wrap)) % (1 << ell))
    return np.array(out, dtype=object)
