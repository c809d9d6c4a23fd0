"""Philox4x32-10 counter-based generator (oracle side; test infrastructure only).

Written from its published definition (J. K. Salmon, M. A. Moraes, R. O. Dror,
D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter
and a 2 x 32-bit key; each of the 10 rounds multiplies counter words 0 and 2 by the two
round multipliers, takes the 64-bit products apart into high and low halves, and
permutes/xors them with words 1 and 3 and the key; the key is bumped by the two Weyl
constants between rounds.

This module is independent of the device implementation; the two agree bit for bit
(the known-answer vectors of the generator pin this one).
"""

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: 4 uint32-valued arrays (broadcastable), key: 2 uint32-valued arrays.
    Returns 4 uint32 arrays (as uint64 dtype holding 32-bit values)."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & _MASK for k in key)
    for r in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if r < 9:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def uniform01(word):
    """u = (r + 1/2) 2^-32 in (0, 1); exact in FP64 for every 32-bit r."""
    return (np.asarray(word, dtype=np.float64) + 0.5) * (2.0 ** -32)
