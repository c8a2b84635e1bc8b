"""Plain CPU oracle of the Bicoptor 2.0 share-local DReLU/ReLU pipeline.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
header, table or constant generator with the HIP library under
``paper_2309_04909_amd/``, and it imports nothing from there.

Everything is exact integer arithmetic on NumPy ``uint64`` arrays (Python
integers where a product exceeds 64 bits), vectorised over elements and
looping over window positions, written to be checked against the paper by
eye.  Module map:

* ``ring``       -- Z_{2^l} helpers (Notations and the cut function, Sec. 2.2-2.3).
* ``params``     -- the prime p (bit length l_x + 1, Tab. 2), parameter checks,
                    the key-bit window (Sec. 6.1).
* ``protocols``  -- Alg. 1 (SecureML truncation), Alg. 4/5 (deterministic
                    truncation), Alg. 6 (modulo switch), Alg. 7 (DReLU) also
                    with the parties apart (packed round-1 messages), Alg. 8
                    (UBL ReLU), Alg. drelu2 and the RSS ReLU (replicated
                    sharing), Alg. linear (truncate-then-multiply) and
                    multiply-then-truncate, message accounting (Tab. 1).
* ``philox``     -- Philox4x32-10 (Salmon et al., SC'11) and the draws that
                    turn its words into t, the shuffle, r_i, z_i, rho, the
                    Beaver triples and the replicated-sharing values.  The
                    paper fixes no PRG for the seeded draws; this module is
                    the build's definition of them.

Pins (what ties each part to the paper rather than to itself) live in
``tests/test_oracle_*.py``.  The Philox4x32-10 function is pinned against
an independent implementation, rocRAND's header-only engine (every counter
and key word), and by statistical and structural properties; no published
known-answer vector is available in this environment.
"""

from . import ring, params, protocols, philox  # noqa: F401
