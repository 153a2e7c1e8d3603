"""Counter-based random numbers for the seeded synthetic inputs.

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 128-bit counter and a 64-bit key are mixed by ten
rounds of two 32x32->64 multiplies; the key is bumped by the Weyl constants
between rounds.  Written from that definition; vectorised over counters.

This module produces INPUTS only.  It holds none of the G4 accumulation's
arithmetic; the oracle and the HIP library both consume what it (or the
library's device twin of the same published generator) produces.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds.  Counter words c0..c3 and key words k0, k1 are
    uint32 arrays (broadcastable).  Returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.asarray(k0, dtype=np.uint32)
    k1 = np.asarray(k1, dtype=np.uint32)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for r in range(10):
        if r:
            k0 = ((k0.astype(np.uint64) + np.uint64(_W0)) & _MASK32).astype(np.uint32)
            k1 = ((k1.astype(np.uint64) + np.uint64(_W1)) & _MASK32).astype(np.uint32)
        p0 = _M0 * c0.astype(np.uint64)
        p1 = _M1 * c2.astype(np.uint64)
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & _MASK32).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & _MASK32).astype(np.uint32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def u53(a, b):
    """Uniform double in [0, 1) from two uint32 words (27 + 26 high bits)."""
    a = np.asarray(a, dtype=np.uint32) >> np.uint32(5)
    b = np.asarray(b, dtype=np.uint32) >> np.uint32(6)
    return (a.astype(np.float64) * 67108864.0 + b.astype(np.float64)) * (1.0 / 9007199254740992.0)


def box_muller(u1, u2):
    """Two independent N(0,1) values from two uniforms in [0,1);
    1-u1 lies in (0,1] so the logarithm is finite."""
    rad = np.sqrt(-2.0 * np.log1p(-u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)
