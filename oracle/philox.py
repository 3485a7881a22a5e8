"""Oracle: Philox4x32-10 counter-based generator (test infrastructure only).

Written from its published definition (J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): four 32-bit counter words, two 32-bit key words, ten rounds; each
round multiplies counter words 0 and 2 by the two Philox multipliers, and
mixes the high halves with the other counter words and the round key; the key
is advanced by the two Weyl constants between rounds.

Parity: pinned by the published known-answer vectors in
tests/test_oracle_philox_sampler.py.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ctr = 4 uint32 words, key = 2 uint32 words -> 4 uint32 words.

    Vectorised: each argument entry may be a numpy array (broadcast together).
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & MASK for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))
