"""Low-rank truncation of a basis vector viewed as an image: tau_r and its
randomized-SVD variant.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

Definitions followed:
  * tau_r (Sec. 1.2, eq. (def:lowr-trc)): reshape the vector c into the 2D array
    C, replace C by its rank-r truncated SVD C_r = U_r Sigma_r V_r^T, and
    vectorise back.  Used as the flexible operator z_k = tau(p_k) of eq. (FGK)
    by FLSQR, sFLSQR and sFLSMR in the deblurring experiments (Sec. 3.1).
  * the "-RND" solvers of Sec. 3.1 replace the truncated SVD by the randomized
    SVD of Halko, Martinsson and Tropp (SIAM Review 53, 2011): randomized
    subspace iteration (their Algorithm 4.4) for an orthonormal Q whose range
    approximates that of C, then the SVD of B = Q^T C (their Algorithm 5.1),
    truncated to rank r.

Readings where the paper is silent (listed in the design notes):
  * vec is the row-major order of the image (pixel (i, j) at i * nc + j).  The
    paper stacks columns; since (C^T)_r = (C_r)^T, both orders give the same
    tau_r;
  * r >= min(nr, nc) leaves the vector unchanged; so does the zero vector;
  * randomized variant: oversampling p = 10 and q = 1 power iteration unless
    given (the paper does not state them); l = min(r + p, nr, nc) test vectors;
  * the test matrix Omega (nc x l) has independent N(0, 1) entries, drawn for
    each call: entry e = j * nc + i (column j, row i) is normal (e mod 4) of the
    Philox4x64-10 block with counter (call, e >> 2, 0, 0) and key (seed,
    2 + (instance << 32)); the block's words (w0, w1) and (w2, w3) give two
    normals each by the Box-Muller transform of u1 = (w_even >> 11 + 1/2) 2^-53
    and u2 = (w_odd >> 11) 2^-53: sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
    'call' is the index k of the basis vector p_k being truncated (1, 2, ...).
"""
from __future__ import annotations

import numpy as np

from . import philox

STREAM_LOWRANK = 2


def as_image(c: np.ndarray, nr: int, nc: int) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64)
    if c.shape != (nr * nc,):
        raise ValueError(f"vector of length {c.shape} is not a {nr} x {nc} image")
    return c.reshape(nr, nc)


def truncate(c: np.ndarray, nr: int, nc: int, r: int) -> np.ndarray:
    """tau_r(c) of eq. (def:lowr-trc) through the full SVD (LAPACK)."""
    C = as_image(c, nr, nc)
    if r >= min(nr, nc):
        return C.ravel().copy()
    U, s, Vt = np.linalg.svd(C, full_matrices=False)
    return ((U[:, :r] * s[:r]) @ Vt[:r]).ravel()


def gaussian_test_matrix(nc: int, l: int, seed: int, call: int, instance: int = 0) -> np.ndarray:
    """Omega (nc x l), N(0, 1) entries from Philox4x64-10 by Box-Muller (see the
    module header for the counter layout)."""
    total = nc * l
    nblk = (total + 3) // 4
    key = (int(seed) & philox.MASK64,
           (STREAM_LOWRANK + (int(instance) << 32)) & philox.MASK64)
    w = philox.blocks(np.uint64(call), np.arange(nblk, dtype=np.uint64), np.uint64(0),
                      np.uint64(0), key)
    two53 = 2.0 ** -53
    out = np.empty((nblk, 4))
    for pair in range(2):
        u1 = ((w[2 * pair] >> np.uint64(11)).astype(np.float64) + 0.5) * two53
        u2 = (w[2 * pair + 1] >> np.uint64(11)).astype(np.float64) * two53
        rad = np.sqrt(-2.0 * np.log(u1))
        ang = 2.0 * np.pi * u2
        out[:, 2 * pair] = rad * np.cos(ang)
        out[:, 2 * pair + 1] = rad * np.sin(ang)
    flat = out.ravel()[:total]
    return flat.reshape(l, nc).T            # entry e = j * nc + i -> Omega[i, j]


def _orth(Y: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def randomized_truncate(c: np.ndarray, nr: int, nc: int, r: int, *, p: int = 10, q: int = 1,
                        seed: int = 0, call: int = 1, instance: int = 0,
                        omega: np.ndarray | None = None) -> np.ndarray:
    """Rank-r truncation through the randomized SVD (HMT Algorithms 4.4 and 5.1)."""
    C = as_image(c, nr, nc)
    if r >= min(nr, nc):
        return C.ravel().copy()
    l = min(r + p, nr, nc)
    Om = gaussian_test_matrix(nc, l, seed, call, instance) if omega is None else omega
    Q = _orth(C @ Om)                       # range finder on Y = C Omega
    for _ in range(q):                      # power iterations, re-orthonormalised
        Q = _orth(C.T @ Q)
        Q = _orth(C @ Q)
    Bm = Q.T @ C                            # l x nc
    Ub, s, Vt = np.linalg.svd(Bm, full_matrices=False)
    U = Q @ Ub
    return ((U[:, :r] * s[:r]) @ Vt[:r]).ravel()


class Truncation:
    """tau_r as a flexible operator for fgk: z_k = tau_r(p_k)."""

    def __init__(self, nr: int, nc: int, r: int):
        self.nr, self.nc, self.r = nr, nc, r

    def __call__(self, p: np.ndarray, x_prev: np.ndarray, k: int) -> np.ndarray:
        return truncate(p, self.nr, self.nc, self.r)


class RandomizedTruncation:
    """Randomized tau_r as a flexible operator; the call index is k of p_k."""

    def __init__(self, nr: int, nc: int, r: int, *, p: int = 10, q: int = 1, seed: int = 0,
                 instance: int = 0):
        self.nr, self.nc, self.r, self.p, self.q = nr, nc, r, p, q
        self.seed, self.instance = seed, instance

    def __call__(self, p: np.ndarray, x_prev: np.ndarray, k: int) -> np.ndarray:
        return randomized_truncate(p, self.nr, self.nc, self.r, p=self.p, q=self.q,
                                   seed=self.seed, call=k, instance=self.instance)
