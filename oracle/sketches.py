"""Sketching operators S (s x d) for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The paper names the families only (Sec. 2.7: Gaussian, subsampled trigonometric
transforms, sparse arrays; CountSketch for the imaging experiments; Gaussian
entries N(0, 1) in Corollary 1).  The concrete definitions used here, and by
the GPU path, are:

* sparse-sign with zeta nonzeros per column (zeta = 1 is CountSketch): column
  j holds zeta distinct rows with values +-1/sqrt(zeta).  Rows and signs come
  from Philox4x64-10 with key (seed, stream + (instance << 32)), stream 0, and
  block counters (j, t, 0, 0), t = 0, 1, ...; the four words of each block are
  used in order; a word u proposes row ((u >> 32) * s) >> 32 with sign
  negative iff (u & 1); proposals already taken in the column are skipped.
* SRHT: S v = sqrt(N/s) R H_N D pad(v), N = 2^ceil(log2 d), H_N the Sylvester
  ordered Hadamard matrix with entries (-1)^popcount(r & c) / sqrt(N), D = diag
  of +-1 where D_i is negative iff bit (i mod 64) of word ((i >> 6) & 3) of the
  stream-0 block with counter (i >> 8, 0, 0, 0) is set, and R selects s rows
  of a partial Fisher-Yates shuffle of [0, N): step t swaps positions t and
  t + mulhi64(u_t, N - t), u_t being word (t & 3) of the stream-1 block with
  counter (t >> 2, 0, 0, 0).
* Gaussian (oracle only): dense N(0, 1/s) entries from numpy's PCG64 stream.
* identity: S = I (s = d).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import philox

STREAM_MAIN = 0
STREAM_SRHT_ROWS = 1


def make_key(seed: int, stream: int, instance: int = 0) -> tuple[int, int]:
    return (int(seed) & philox.MASK64, (int(stream) + (int(instance) << 32)) & philox.MASK64)


# ----------------------------------------------------------------------------
# sparse-sign / CountSketch
# ----------------------------------------------------------------------------

def sparse_sign_codes_loop(d: int, s: int, zeta: int, seed: int, instance: int = 0):
    """Plain per-column loop (small d): rows (d, zeta) and signs (d, zeta) in draw order."""
    key = make_key(seed, STREAM_MAIN, instance)
    rows = np.zeros((d, zeta), dtype=np.int64)
    signs = np.zeros((d, zeta), dtype=np.int64)
    for j in range(d):
        taken = []
        tsign = []
        t = 0
        while len(taken) < zeta:
            for u in philox.block((j, t, 0, 0), key):
                if len(taken) == zeta:
                    break
                r = ((u >> 32) * s) >> 32
                if r in taken:
                    continue
                taken.append(r)
                tsign.append(-1 if (u & 1) else 1)
            t += 1
        rows[j] = taken
        signs[j] = tsign
    return rows, signs


def sparse_sign_codes(d: int, s: int, zeta: int, seed: int, instance: int = 0):
    """Vectorised over columns; identical output to sparse_sign_codes_loop."""
    if not (1 <= zeta <= s):
        raise ValueError("need 1 <= zeta <= s")
    key = make_key(seed, STREAM_MAIN, instance)
    rows = np.full((d, zeta), -1, dtype=np.int64)
    signs = np.zeros((d, zeta), dtype=np.int64)
    count = np.zeros(d, dtype=np.int64)
    active = np.arange(d, dtype=np.int64)
    t = 0
    s64 = np.uint64(s)
    while active.size:
        words = philox.blocks(active.astype(np.uint64), np.uint64(t), np.uint64(0), np.uint64(0), key)
        for u in words:
            cand = ((u >> np.uint64(32)) * s64) >> np.uint64(32)
            cand = cand.astype(np.int64)
            sg = np.where((u & np.uint64(1)) != 0, -1, 1)
            cnt = count[active]
            dup = (rows[active] == cand[:, None]).any(axis=1)
            acc = (cnt < zeta) & ~dup
            cols = active[acc]
            rows[cols, cnt[acc]] = cand[acc]
            signs[cols, cnt[acc]] = sg[acc]
            count[cols] += 1
        active = active[count[active] < zeta]
        t += 1
    return rows, signs


class SparseSign:
    """S (s x d) with zeta entries +-1/sqrt(zeta) per column."""

    kind = "sparse_sign"

    def __init__(self, d: int, s: int, zeta: int, seed: int, instance: int = 0):
        self.d, self.s, self.zeta, self.seed = d, s, zeta, seed
        self.rows, self.signs = sparse_sign_codes(d, s, zeta, seed, instance)
        cols = np.repeat(np.arange(d), zeta)
        vals = self.signs.ravel() / math.sqrt(zeta)
        self.S = sp.csr_matrix((vals, (self.rows.ravel(), cols)), shape=(s, d))

    def apply(self, v: np.ndarray) -> np.ndarray:
        return self.S @ v

    def matrix(self) -> np.ndarray:
        return self.S.toarray()


# ----------------------------------------------------------------------------
# SRHT
# ----------------------------------------------------------------------------

def next_pow2(d: int) -> int:
    N = 1
    while N < d:
        N *= 2
    return N


def fwht(x: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform in Sylvester order: H x,
    H[r, c] = (-1)^popcount(r & c).  Uses H_2h = [[H_h, H_h], [H_h, -H_h]]."""
    N = x.shape[0]
    y = np.array(x, dtype=np.float64, copy=True)
    h = 1
    while h < N:
        y = y.reshape(-1, 2, h)
        a = y[:, 0, :].copy()
        b = y[:, 1, :].copy()
        y = np.stack([a + b, a - b], axis=1).reshape(N)
        h *= 2
    return y


def srht_signs(N: int, seed: int, instance: int = 0) -> np.ndarray:
    """D as +-1 array of length N."""
    key = make_key(seed, STREAM_MAIN, instance)
    nblk = (N + 255) // 256
    words = philox.blocks(np.arange(nblk, dtype=np.uint64), np.uint64(0), np.uint64(0),
                          np.uint64(0), key)
    W = np.stack(words, axis=1)                                 # (nblk, 4)
    i = np.arange(N, dtype=np.int64)
    word = W[i >> 8, (i >> 6) & 3]
    bit = (word >> (i & 63).astype(np.uint64)) & np.uint64(1)
    return np.where(bit != 0, -1.0, 1.0)


def srht_rows(N: int, s: int, seed: int, instance: int = 0) -> np.ndarray:
    """s distinct rows of [0, N) from a partial Fisher-Yates shuffle."""
    if not (1 <= s <= N):
        raise ValueError("need 1 <= s <= N")
    key = make_key(seed, STREAM_SRHT_ROWS, instance)
    perm = list(range(N))
    blk = None
    for t in range(s):
        if t % 4 == 0:
            blk = philox.block((t >> 2, 0, 0, 0), key)
        u = blk[t & 3]
        j = t + philox.mulhi64(u, N - t)
        perm[t], perm[j] = perm[j], perm[t]
    return np.array(perm[:s], dtype=np.int64)


class SRHT:
    """S v = sqrt(N/s) R H_N D pad(v) with normalised H_N."""

    kind = "srht"

    def __init__(self, d: int, s: int, seed: int, instance: int = 0):
        self.d, self.s, self.seed = d, s, seed
        self.N = next_pow2(d)
        self.D = srht_signs(self.N, seed, instance)
        self.rows = srht_rows(self.N, s, seed, instance)

    def apply(self, v: np.ndarray) -> np.ndarray:
        u = np.zeros(self.N)
        u[: self.d] = v
        Hu = fwht(self.D * u) / math.sqrt(self.N)
        return math.sqrt(self.N / self.s) * Hu[self.rows]

    def matrix(self) -> np.ndarray:
        return np.stack([self.apply(e) for e in np.eye(self.d)], axis=1)


# ----------------------------------------------------------------------------
# Gaussian and identity
# ----------------------------------------------------------------------------

class Gaussian:
    kind = "gaussian"

    def __init__(self, d: int, s: int, seed: int):
        self.d, self.s = d, s
        self.G = np.random.default_rng(seed).standard_normal((s, d)) / math.sqrt(s)

    def apply(self, v):
        return self.G @ v

    def matrix(self):
        return self.G


class Identity:
    kind = "identity"

    def __init__(self, d: int):
        self.d = self.s = d

    def apply(self, v):
        return np.array(v, dtype=np.float64, copy=True)

    def matrix(self):
        return np.eye(self.d)


class Dense:
    """An arbitrary explicit sketch matrix (used for the Remark equivalence)."""
    kind = "dense"

    def __init__(self, M: np.ndarray):
        self.M = np.asarray(M, dtype=np.float64)
        self.s, self.d = self.M.shape

    def apply(self, v):
        return self.M @ v

    def matrix(self):
        return self.M


def make(kind: str, d: int, s: int, seed: int, zeta: int = 8, instance: int = 0):
    if kind == "sparse_sign":
        return SparseSign(d, s, zeta, seed, instance)
    if kind == "countsketch":
        return SparseSign(d, s, 1, seed, instance)
    if kind == "srht":
        return SRHT(d, s, seed, instance)
    if kind == "gaussian":
        return Gaussian(d, s, seed)
    if kind == "identity":
        return Identity(d)
    raise ValueError(kind)
