"""Philox4x32-10 counter-based generator, written from its published definition.

Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11), Section 4: a 4x32-bit counter and a 2x32-bit key; each of the 10
rounds multiplies words 0 and 2 by fixed odd constants, swaps and XORs the
high halves with the other words and the key, and the key is bumped by the two
Weyl constants between rounds.

Pinned by the paper's / Random123's known-answer vectors (tests/golden).
Vectorised over arrays of counters with uint64 products.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Return the four 32-bit output words for counters (c0..c3) under key (k0, k1).

    Counter words may be numpy arrays (broadcast together); results are uint32.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    ka = int(k0) & 0xFFFFFFFF
    kb = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(ka), lo1, hi0 ^ c3 ^ np.uint64(kb), lo0)
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32),
            c3.astype(np.uint32))
