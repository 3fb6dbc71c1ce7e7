"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), vectorised in numpy.

This module holds no arithmetic of the fitting method: it only turns
(counter, key) pairs into uniformly distributed bits.  Everything is uint64
numpy arithmetic so that 32x32->64 products are exact.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32(ctr, key, rounds: int = 10):
    """Apply Philox4x32 with `rounds` rounds.

    ctr: four uint32-valued arrays (broadcastable); key: two uint32 values or
    arrays.  Returns a tuple of four uint64 arrays holding 32-bit words.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & _MASK for k in key)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    for r in range(rounds):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniforms(n: int, key, stream: int, word: int = 0):
    """Two arrays of n uniforms in [0, 1) from counters
    (i mod 2^32, i >> 32, stream, word), i = 0..n-1.

    Each Philox output (4 words) yields two 53-bit doubles
    u = (hi:lo >> 11) * 2^-53 with hi the first word of each pair.
    """
    i = np.arange(n, dtype=np.uint64)
    return uniforms_at(i, key, stream, word)


def uniforms_at(i, key, stream: int, word: int = 0):
    """Two uniforms per counter index array `i` (see `uniforms`)."""
    i = np.asarray(i, dtype=np.uint64)
    lo_i = i & _MASK
    hi_i = i >> _S32
    r0, r1, r2, r3 = philox4x32((lo_i, hi_i, np.uint64(stream), np.uint64(word)), key)
    a = ((r0 << _S32) | r1) >> np.uint64(11)
    b = ((r2 << _S32) | r3) >> np.uint64(11)
    scale = 2.0 ** -53
    return a.astype(np.float64) * scale, b.astype(np.float64) * scale


def key_from_seed(seed: int, fit: int = 0):
    """Philox key for a base seed and a fit index: (seed mod 2^32, fit)."""
    return (np.uint64(seed & 0xFFFFFFFF), np.uint64(fit & 0xFFFFFFFF))
