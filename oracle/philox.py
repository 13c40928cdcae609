"""Philox4x32-10 counter-based generator (test infrastructure; see oracle/__init__).

Written from the published definition: J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11.  A 4-word counter and a 2-word key go through 10 rounds; each round
multiplies words 0 and 2 by two fixed odd constants, takes the 64-bit
products' high and low halves, XORs the high halves with the other counter
words and the key, and permutes; the key is bumped by two Weyl constants
between rounds.

Pinned by the known-answer vectors of the reference implementation
(tests/test_oracle_sampling.py).
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
ROUNDS = 10


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = ROUNDS):
    """Vectorised Philox4x32: every argument broadcasts; returns 4 uint32 arrays."""
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]          # < 2^64: exact in uint64
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return tuple(v.astype(np.uint32) for v in c)


def u01(word) -> np.ndarray:
    """uint32 -> float32 in [0, 1): the top 24 bits times 2^-24 (exact)."""
    w = np.asarray(word, dtype=np.uint32)
    return ((w >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
