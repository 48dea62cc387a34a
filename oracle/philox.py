"""Philox4x32-10 and the Gaussian noise stream of the Langevin update.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a
multiply/xor S-box on a 128-bit counter under a 64-bit key, the key bumped by
the Weyl constants between rounds.  Written here from that definition.

The Langevin noise eta ~ N(0, 1) (Sec. 3.2, SGLD and eq:pSGLD) is drawn per
(catalog stream, chain, step, event): two Philox blocks per event give four
32-bit words each; each pair of words makes one 52-bit uniform in (0, 1), and
Box-Muller turns two uniforms into two normals.  Block 0 gives (x, y), block 1
gives (z, t).
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85

TAG_NOISE = 1 << 28
TAG_PERM = 2 << 28


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox4x32 rounds on counters (c0..c3, broadcastable uint32 arrays)
    under key (k0, k1).  Returns four uint64 arrays holding the 32-bit outputs."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 &= 0xFFFFFFFF
    k1 &= 0xFFFFFFFF
    for rnd in range(10):
        p0 = _M0 * c0            # 32 x 32 -> 64 bit products, exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        if rnd < 9:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def key_of(seed: int):
    """The 64-bit run seed split into the Philox key words (low, high)."""
    seed &= (1 << 64) - 1
    return seed & 0xFFFFFFFF, seed >> 32


def uniform52(a, b):
    """Two 32-bit words -> one double in (0, 1): the top 26 bits of each word
    form k in [0, 2^52), and u = (k + 1/2) 2^-52, exact in float64, so that
    0 and 1 never occur."""
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    hi = (a >> np.uint64(6)).astype(np.float64)
    lo = (b >> np.uint64(6)).astype(np.float64)
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 4503599627370496.0)


def box_muller(u1, u2):
    """Two independent uniforms -> two independent standard normals."""
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang), r * np.sin(ang)


def noise(seed: int, stream: int, chain: int, step: int, events) -> np.ndarray:
    """eta for the given events at (stream, chain, step): array [len(events), 4]."""
    k0, k1 = key_of(seed)
    m = np.asarray(events, np.uint64)
    out = np.empty((m.shape[0], 4))
    for sub in range(2):
        w = philox4x32_10(m, step & 0xFFFFFFFF, chain, TAG_NOISE | (stream << 4) | sub, k0, k1)
        g0, g1 = box_muller(uniform52(w[0], w[1]), uniform52(w[2], w[3]))
        out[:, 2 * sub] = g0
        out[:, 2 * sub + 1] = g1
    return out
