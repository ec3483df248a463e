"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC 2011), written from its published definition in plain Python integers.

TEST INFRASTRUCTURE ONLY (part of the oracle).  The GPU library implements the same published
generator on its own; the two share no code.

One round maps (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
and the key is bumped by the Weyl constants (W0, W1) between rounds; ten rounds.

Draws used by k-means++ seeding, round m (m = 0, 1, ...), key = (seed mod 2^32, seed >> 32):
* counter (m, 0, 0, 0); the first output word w is used;
* a uniform in [0, 1) with 24 random bits: (w >> 8) * 2^-24 (exact in float32 and float64);
* an index in [0, n): (w * n) >> 32.
"""
from __future__ import annotations

_MASK = 0xFFFFFFFF
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(counter, key):
    c0, c1, c2, c3 = (int(v) & _MASK for v in counter)
    k0, k1 = (int(v) & _MASK for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & _MASK
            k1 = (k1 + W1) & _MASK
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & _MASK, p1 & _MASK, \
                         ((p0 >> 32) ^ c3 ^ k1) & _MASK, p0 & _MASK
    return c0, c1, c2, c3


def _word(seed: int, m: int) -> int:
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return philox4x32_10((m, 0, 0, 0), (seed & _MASK, seed >> 32))[0]


def philox_uniform24(seed: int, m: int) -> float:
    return (_word(seed, m) >> 8) * 2.0 ** -24


def philox_index(seed: int, m: int, n: int) -> int:
    return (_word(seed, m) * int(n)) >> 32
