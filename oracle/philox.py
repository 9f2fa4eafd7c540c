"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from its published definition.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The paper leaves the random generator of its sketches unspecified (Sec. 2.7
only names the sketch families).  Both the GPU path and this oracle derive the
sketch from a seed with this counter-based generator, so that indices and signs
can be compared bit for bit.

Block function: state (x0, x1, x2, x3) and key (k0, k1); ten rounds of
    (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2          (128-bit products)
    x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
with the key bumped by the Weyl constants (W0, W1) between rounds.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
ROUNDS = 10


def block(ctr, key):
    """One Philox4x64-10 block with Python integers: 4 words out."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(ROUNDS):
        if r > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK64, (p0 >> 64) ^ x3 ^ k1, p0 & MASK64)
    return (x0, x1, x2, x3)


_U32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: int):
    """(hi, lo) of the 128-bit product of uint64 arrays a and constant b."""
    b = np.uint64(b)
    a0, a1 = a & _U32, a >> _S32
    b0, b1 = b & _U32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _U32) + (p10 & _U32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def blocks(c0, c1, c2, c3, key):
    """Vectorised block function over uint64 counter arrays; returns 4 arrays."""
    with np.errstate(over="ignore"):
        x0 = np.asarray(c0, dtype=np.uint64).copy()
        x1 = np.asarray(c1, dtype=np.uint64).copy()
        x2 = np.asarray(c2, dtype=np.uint64).copy()
        x3 = np.asarray(c3, dtype=np.uint64).copy()
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        x0, x1, x2, x3 = x0.copy(), x1.copy(), x2.copy(), x3.copy()
        k0 = int(key[0]) & MASK64
        k1 = int(key[1]) & MASK64
        for r in range(ROUNDS):
            if r > 0:
                k0 = (k0 + W0) & MASK64
                k1 = (k1 + W1) & MASK64
            hi0, lo0 = _mulhilo(x0, M0)
            hi1, lo1 = _mulhilo(x2, M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0
    return x0, x1, x2, x3


def mulhi64(u: int, n: int) -> int:
    """floor(u * n / 2^64): maps a uniform 64-bit word to [0, n)."""
    return (int(u) * int(n)) >> 64
