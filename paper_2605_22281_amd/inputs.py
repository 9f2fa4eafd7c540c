"""Seeded synthetic inputs for the sketched flexible LSQR/LSMR solvers.

This module builds test problems only: phantoms, 2D parallel-beam projection
matrices, an unmatched pixel-driven back-projector, noise, the artificial
ill-posed matrices of the paper's synthetic experiment, and the Gaussian
blur + subsampling operator of its deblurring and inpainting example.  It contains none of the
solver's arithmetic and serves both the CPU oracle and the GPU path, which each
receive the same arrays.

Problem model (paper, Section 1, eq. (inverseproblem)): b = A x_true + e with
white Gaussian e scaled to a prescribed noise level delta = ||e|| / ||A x_true||.

Geometry conventions (the paper's CT matrices come from ASTRA, which is not
available; these are the stand-ins):
  * image of N x N unit pixels covering [-N/2, N/2]^2, vectorised row-major,
    pixel (r, c) covering x in [c - N/2, c - N/2 + 1], y in [r - N/2, r - N/2 + 1];
  * angles theta_a = a * pi / N_a, a = 0..N_a-1 (equispaced in [0, pi));
  * N_d detector bins of unit width, centred: t_d = d - (N_d - 1) / 2;
  * ray (a, d) is {p : p . u_a = t_d} with u_a = (cos theta_a, sin theta_a); its
    matrix row index is a * N_d + d;
  * A[ray, pixel] = exact length of the ray inside the pixel (Siddon's method);
    a segment lying on a grid line goes to the pixel containing its midpoint;
  * B (unmatched back-projector, n x m): pixel-driven linear interpolation.  For
    pixel centre c and angle a the continuous bin coordinate is
    u = c . u_a + (N_d - 1) / 2; weights (1 - f, f) go to bins floor(u) and
    floor(u) + 1 with f = u - floor(u); bins outside [0, N_d) are dropped.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np
import scipy.sparse as sp

# Seed bases per workload item; instance i of a batch adds INSTANCE_STRIDE * i.
SEED_PHANTOM = 1000
SEED_NOISE = 2000
SEED_SKETCH = 3000
INSTANCE_STRIDE = 100000


# ----------------------------------------------------------------------------
# Projection geometry
# ----------------------------------------------------------------------------

def geometry_for_side(side: int) -> tuple[int, int]:
    """Angles and detector bins used for an image of the given side.

    N_a = round(0.7 * side), N_d = ceil(sqrt(2) * side).  The detector rule also
    reproduces the 91 / 363 / 725 bins of the 64^2 / 256^2 / 512^2 workloads,
    whose angle counts (90 / 180 / 360) are fixed explicitly instead.
    """
    return int(round(0.7 * side)), int(math.ceil(math.sqrt(2.0) * side))


@functools.lru_cache(maxsize=8)
def siddon_matrix(N: int, n_angles: int, n_det: int, chunk_rays: int = 16384) -> sp.csr_matrix:
    """Exact ray/pixel intersection lengths, CSR (m = n_angles * n_det, n = N * N).

    Rows are sorted by column index; int32 indices; float64 values.
    """
    m = n_angles * n_det
    half = N / 2.0
    grid = np.arange(N + 1, dtype=np.float64) - half          # grid line coordinates
    theta = np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)
    t_det = np.arange(n_det, dtype=np.float64) - (n_det - 1) / 2.0

    indptr = np.zeros(m + 1, dtype=np.int64)
    cols_parts, vals_parts = [], []
    ray0 = 0
    while ray0 < m:
        ray1 = min(m, ray0 + chunk_rays)
        rid = np.arange(ray0, ray1)
        a = rid // n_det
        d = rid % n_det
        ux, uy = np.cos(theta[a]), np.sin(theta[a])
        vx, vy = -uy, ux                                      # ray direction, unit length
        t = t_det[d]
        ox, oy = t * ux, t * uy                               # point of the ray closest to 0
        big = 4.0 * N
        with np.errstate(divide="ignore", invalid="ignore"):
            lx = (grid[None, :] - ox[:, None]) / vx[:, None]
            ly = (grid[None, :] - oy[:, None]) / vy[:, None]
        # clip interval: where the ray is inside the square
        okx = np.abs(vx) > 1e-15
        oky = np.abs(vy) > 1e-15
        lxmin = np.where(okx, np.minimum(lx[:, 0], lx[:, -1]), -big)
        lxmax = np.where(okx, np.maximum(lx[:, 0], lx[:, -1]), big)
        lymin = np.where(oky, np.minimum(ly[:, 0], ly[:, -1]), -big)
        lymax = np.where(oky, np.maximum(ly[:, 0], ly[:, -1]), big)
        # rays parallel to an axis must lie within the square's extent
        inside_x = okx | ((ox >= -half) & (ox <= half))
        inside_y = oky | ((oy >= -half) & (oy <= half))
        lmin = np.maximum(lxmin, lymin)
        lmax = np.minimum(lxmax, lymax)
        valid_ray = inside_x & inside_y & (lmax > lmin)
        lx = np.where(okx[:, None], lx, np.nan)
        ly = np.where(oky[:, None], ly, np.nan)
        lam = np.concatenate([lx, ly, lmin[:, None], lmax[:, None]], axis=1)
        lam = np.where((lam >= lmin[:, None]) & (lam <= lmax[:, None]), lam, np.nan)
        lam.sort(axis=1)                                      # NaNs go last
        seg = lam[:, 1:] - lam[:, :-1]
        mid = 0.5 * (lam[:, 1:] + lam[:, :-1])
        good = np.isfinite(seg) & (seg > 1e-9) & valid_ray[:, None]
        xm = ox[:, None] + mid * vx[:, None]
        ym = oy[:, None] + mid * vy[:, None]
        with np.errstate(invalid="ignore"):
            ci = np.floor(xm + half)
            ri = np.floor(ym + half)
        good &= (ci >= 0) & (ci < N) & (ri >= 0) & (ri < N)
        counts = good.sum(axis=1)
        pix = (ri[good] * N + ci[good]).astype(np.int64)
        lens = seg[good]
        # sort each ray's entries by pixel index
        rowid = np.repeat(np.arange(ray1 - ray0), counts)
        order = np.lexsort((pix, rowid))
        cols_parts.append(pix[order].astype(np.int32))
        vals_parts.append(lens[order])
        indptr[ray0 + 1:ray1 + 1] = counts
        ray0 = ray1
    indptr = np.cumsum(indptr)
    cols = np.concatenate(cols_parts) if cols_parts else np.zeros(0, np.int32)
    vals = np.concatenate(vals_parts) if vals_parts else np.zeros(0)
    A = sp.csr_matrix((vals, cols, indptr.astype(np.int64)), shape=(m, N * N))
    return _as_int32_csr(A)


@functools.lru_cache(maxsize=4)
def pixel_driven_backprojector(N: int, n_angles: int, n_det: int) -> sp.csr_matrix:
    """Unmatched back-projector B (n x m), linear interpolation between bins."""
    n = N * N
    half = N / 2.0
    theta = np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)
    r = np.arange(N, dtype=np.float64)
    yc = (r - half + 0.5)[:, None] * np.ones((1, N))
    xc = np.ones((N, 1)) * (r - half + 0.5)[None, :]
    xc = xc.ravel()
    yc = yc.ravel()
    rows_parts, cols_parts, vals_parts = [], [], []
    pix = np.arange(n, dtype=np.int64)
    for a in range(n_angles):
        u = xc * math.cos(theta[a]) + yc * math.sin(theta[a]) + (n_det - 1) / 2.0
        lo = np.floor(u)
        f = u - lo
        lo = lo.astype(np.int64)
        for bins, w in ((lo, 1.0 - f), (lo + 1, f)):
            keep = (bins >= 0) & (bins < n_det) & (w > 0.0)
            rows_parts.append(pix[keep])
            cols_parts.append(a * n_det + bins[keep])
            vals_parts.append(w[keep])
    rows = np.concatenate(rows_parts)
    cols = np.concatenate(cols_parts)
    vals = np.concatenate(vals_parts)
    B = sp.csr_matrix((vals, (rows, cols)), shape=(n, n_angles * n_det))
    B.sum_duplicates()
    B.sort_indices()
    return _as_int32_csr(B)


def _as_int32_csr(M: sp.spmatrix) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    M.sort_indices()
    if M.nnz >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    M.indptr = M.indptr.astype(np.int32)
    M.indices = M.indices.astype(np.int32)
    M.data = M.data.astype(np.float64)
    return M


# ----------------------------------------------------------------------------
# Phantoms and noise
# ----------------------------------------------------------------------------

def ellipse_phantom(N: int, seed: int, n_ellipses: int = 6) -> np.ndarray:
    """Sum of random ellipses (additive overlap), row-major length N*N.

    Centres U[-0.5, 0.5]^2 and semi-axes U[0.1, 0.5] in units of the half-width,
    rotation U[0, pi), intensity U[0.2, 1]; a pixel belongs to an ellipse when
    its centre does.
    """
    rng = np.random.default_rng(seed)
    half = N / 2.0
    coords = (np.arange(N) - half + 0.5) / half               # pixel centres in [-1, 1]
    Y, X = np.meshgrid(coords, coords, indexing="ij")
    img = np.zeros((N, N))
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.5, 0.5, size=2)
        ax, ay = rng.uniform(0.1, 0.5, size=2)
        phi = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.2, 1.0)
        c, s = math.cos(phi), math.sin(phi)
        xr = (X - cx) * c + (Y - cy) * s
        yr = -(X - cx) * s + (Y - cy) * c
        img += val * ((xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0)
    return img.ravel()


def sparse_phantom(N: int, seed: int, fraction: float = 0.02) -> np.ndarray:
    """A fraction of pixels (chosen without replacement) set to U[0, 1]."""
    rng = np.random.default_rng(seed)
    n = N * N
    k = int(round(fraction * n))
    x = np.zeros(n)
    idx = rng.choice(n, size=k, replace=False)
    x[idx] = rng.uniform(0.0, 1.0, size=k)
    return x


def add_noise(b_true: np.ndarray, level: float, seed: int) -> tuple[np.ndarray, float]:
    """b = b_true + e with ||e|| = level * ||b_true|| exactly; returns (b, ||e||)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(b_true.shape[0])
    e = level * np.linalg.norm(b_true) * g / np.linalg.norm(g)
    return b_true + e, float(np.linalg.norm(e))


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One least-squares problem min ||A x - b|| with its ground truth."""
    A: sp.csr_matrix
    B: sp.csr_matrix | None          # None means B = A^T (matched transpose)
    b: np.ndarray
    x_true: np.ndarray
    noise_norm: float                # delta_e = ||e||
    N: int = 0
    n_angles: int = 0
    n_det: int = 0
    name: str = ""

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    def backprojector(self) -> sp.csr_matrix:
        return self.B if self.B is not None else _as_int32_csr(self.A.T.tocsr())


def ct_problem(N: int, n_angles: int, n_det: int, *, phantom: str = "ellipses",
               noise: float = 0.01, seed_offset: int = 0, unmatched: bool = False,
               name: str = "") -> Problem:
    A = siddon_matrix(N, n_angles, n_det)
    if phantom == "ellipses":
        x = ellipse_phantom(N, SEED_PHANTOM + seed_offset)
    elif phantom == "sparse":
        x = sparse_phantom(N, SEED_PHANTOM + seed_offset)
    else:
        raise ValueError(phantom)
    b, dn = add_noise(A @ x, noise, SEED_NOISE + seed_offset)
    B = pixel_driven_backprojector(N, n_angles, n_det) if unmatched else None
    return Problem(A=A, B=B, b=b, x_true=x, noise_norm=dn, N=N, n_angles=n_angles,
                   n_det=n_det, name=name)


# The workloads (64^2 / 256^2 / 512^2 images, heterogeneous batch).
WORKLOADS = {
    "ct64": dict(N=64, n_angles=90, n_det=91, phantom="ellipses", noise=0.01, seed_offset=1),
    "ct256_unmatched": dict(N=256, n_angles=180, n_det=363, phantom="ellipses", noise=0.02,
                            seed_offset=2, unmatched=True),
    "ct512_sparse": dict(N=512, n_angles=360, n_det=725, phantom="sparse", noise=0.01,
                         seed_offset=3),
}


def workload(name: str) -> Problem:
    if name in DEBLUR_WORKLOADS:
        return deblur_problem(name=name, **DEBLUR_WORKLOADS[name])
    kw = dict(WORKLOADS[name])
    return ct_problem(name=name, **kw)


# ----------------------------------------------------------------------------
# Deblurring and inpainting (paper, Sec. 1.2 motivating example and Sec. 3.1)
# ----------------------------------------------------------------------------

def house_phantom(N: int) -> np.ndarray:
    """A synthetic stand-in for the paper's 'house' photograph (not available):
    a sky with a vertical gradient, a wall, two windows and a door (axis-aligned
    blocks: each is a rank-one image) and a triangular roof, so that the
    singular values decay quickly but the image is not exactly low rank.
    Row-major, values in [0, 1]."""
    y = (np.arange(N) + 0.5) / N
    img = np.repeat((0.3 + 0.4 * y)[:, None], N, axis=1)

    def block(r0, r1, c0, c1, v):
        img[int(r0 * N):int(r1 * N), int(c0 * N):int(c1 * N)] = v

    block(0.45, 0.95, 0.15, 0.85, 0.8)          # wall
    block(0.55, 0.70, 0.25, 0.40, 0.2)          # windows
    block(0.55, 0.70, 0.60, 0.75, 0.2)
    block(0.72, 0.95, 0.45, 0.57, 0.35)         # door
    xc = (np.arange(N) + 0.5) / N
    for i in range(N):
        if 0.15 <= y[i] < 0.45:                 # roof: half-width grows downwards
            h = (y[i] - 0.15) / 0.30 * 0.40
            img[i, np.abs(xc - 0.5) < h] = 0.55
    return img.ravel()


def gaussian_blur_matrix(N: int, variance: float = 0.25, radius: int = 2) -> sp.csr_matrix:
    """Blur by a Gaussian point-spread function of the given variance (pixels^2),
    truncated to a (2 radius + 1)^2 stencil and normalised to unit sum; zero
    boundary conditions.  Separable: K = K1 (x) K1 on the row-major image."""
    off = np.arange(-radius, radius + 1)
    k1 = np.exp(-off.astype(np.float64) ** 2 / (2.0 * variance))
    k1 /= k1.sum()
    K1 = sp.diags([np.full(N - abs(d), k1[d + radius]) for d in off], off, shape=(N, N))
    return sp.kron(K1, K1, format="csr")


def deblur_problem(N: int, *, variance: float = 0.25, keep: float = 0.7, noise: float = 0.05,
                   seed_offset: int = 0, name: str = "") -> Problem:
    """b = M K x + e: Gaussian blur K, then subsampling M that keeps a random
    fraction of the pixels (rows of K; the others are missing), then white noise
    at the relative level 'noise'."""
    rng = np.random.default_rng(SEED_PHANTOM + seed_offset)
    kept = np.sort(rng.choice(N * N, size=int(round(keep * N * N)), replace=False))
    A = _as_int32_csr(gaussian_blur_matrix(N, variance)[kept].tocsr())
    x = house_phantom(N)
    b, dn = add_noise(A @ x, noise, SEED_NOISE + seed_offset)
    return Problem(A=A, B=None, b=b, x_true=x, noise_norm=dn, N=N, name=name)


# The deblurring workloads: 512^2 as in the paper's example (variance 0.25,
# 5% noise); 64^2 for quick tests.
DEBLUR_WORKLOADS = {
    "deblur512": dict(N=512, variance=0.25, keep=0.7, noise=0.05, seed_offset=8),
    "deblur64": dict(N=64, variance=0.25, keep=0.7, noise=0.05, seed_offset=9),
}


def tile_order(N: int, tile: int = 4) -> np.ndarray:
    """An order of the N*N pixels (row-major index j) in tile x tile blocks:
    pixel j goes to position perm[j]; blocks follow each other row-major and
    pixels inside a block row-major (blocks at the edges may be partial).  Rays
    crossing a block then read few consecutive positions in any direction."""
    r, c = np.divmod(np.arange(N * N, dtype=np.int64), N)
    key = ((r // tile) * ((N + tile - 1) // tile) + c // tile) * (tile * tile) + (r % tile) * tile + c % tile
    order = np.argsort(key, kind="stable")          # position -> pixel
    perm = np.empty(N * N, dtype=np.int32)
    perm[order] = np.arange(N * N, dtype=np.int32)  # pixel -> position
    return perm


def batch_instance_sides(count: int = 32, sides=(128, 192, 256, 384), seed: int = 4,
                         max_side: int | None = None) -> list[tuple[int, float]]:
    """(side, noise level) of each instance of batch_instances, without building them."""
    rng = np.random.default_rng(SEED_PHANTOM + seed)
    out = []
    for _ in range(count):
        side = int(rng.choice(sides))
        if max_side is not None:
            side = min(side, max_side)
        out.append((side, float(rng.uniform(0.005, 0.03))))
    return out


def batch_instances(count: int = 32, sides=(128, 192, 256, 384), seed: int = 4,
                    max_side: int | None = None, select=None) -> list[Problem]:
    """Heterogeneous batch: sides drawn uniformly, own phantom, noise U[0.5%, 3%].
    Instances of equal side share the (cached, read-only) projection matrix.
    select: indices of the instances to build (default: all), in that order."""
    drawn = batch_instance_sides(count, sides, seed, max_side)
    out = []
    for i in (range(count) if select is None else select):
        side, level = drawn[i]
        na, nd = geometry_for_side(side)
        out.append(ct_problem(side, na, nd, phantom="ellipses", noise=level,
                              seed_offset=seed + INSTANCE_STRIDE * (i + 1),
                              name=f"batch{i}_side{side}"))
    return out


def multi_rhs(P: Problem, R: int, *, seed: int = 5, noise=None) -> tuple[np.ndarray, np.ndarray,
                                                                         np.ndarray]:
    """R right-hand sides for the operator of P: right-hand side r measures its
    own phantom (ellipses, or sparse like P's if P's phantom is sparse) at its
    own noise level (P's level if noise is None, else noise[r]).  Returns
    (b (R, m), x_true (R, n), noise_norm (R,))."""
    sparse = float(np.mean(P.x_true != 0)) < 0.5
    rel = float(P.noise_norm / np.linalg.norm(P.A @ P.x_true)) if noise is None else None
    bs, xs, dns = [], [], []
    for r in range(R):
        off = seed + INSTANCE_STRIDE * (r + 1)
        x = sparse_phantom(P.N, SEED_PHANTOM + off) if sparse else ellipse_phantom(P.N, SEED_PHANTOM + off)
        bt = P.A @ x
        level = noise[r] if noise is not None else rel
        b, dn = add_noise(bt, level, SEED_NOISE + off)
        bs.append(b)
        xs.append(x)
        dns.append(dn)
    return np.stack(bs), np.stack(xs), np.array(dns)


def small_ct(N: int = 16, n_angles: int = 12, n_det: int | None = None, *, noise: float = 0.01,
             seed_offset: int = 7, unmatched: bool = False, phantom: str = "ellipses") -> Problem:
    """A small CT problem for quick tests."""
    if n_det is None:
        n_det = int(math.ceil(math.sqrt(2.0) * N))
    return ct_problem(N, n_angles, n_det, phantom=phantom, noise=noise,
                      seed_offset=seed_offset, unmatched=unmatched, name=f"ct{N}")


def artificial_problem(m: int = 1024, n: int = 512, rho: float = 1.01, noise: float = 0.01,
                       seed: int = 11) -> Problem:
    """Dense ill-posed test problem of the paper's synthetic experiment (Sec. 2.4).

    A = U diag(rho^(1-i)) V^T with Haar-random orthogonal U (m x n) and V (n x n);
    x_true = ones, b_true = A x_true; x_true and b_true are scaled together so
    that ||b_true|| = 1; then ||e|| = noise (absolute, since ||b_true|| = 1).
    """
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = rho ** (1.0 - np.arange(1, n + 1, dtype=np.float64))
    A = (U * sig[None, :]) @ V.T
    x = np.ones(n)
    bt = A @ x
    scale = 1.0 / np.linalg.norm(bt)
    x *= scale
    bt *= scale
    b, dn = add_noise(bt, noise, seed + 1)
    return Problem(A=_as_int32_csr(sp.csr_matrix(A)), B=None, b=b, x_true=x, noise_norm=dn,
                   name=f"artificial_rho{rho}")


def random_sparse_problem(m: int, n: int, density: float, seed: int, *, unmatched: bool = False,
                          noise: float = 0.01) -> Problem:
    """A generic random sparse problem with a well-conditioned dense part.

    Used for parity tests with ragged row lengths (some rows empty).
    """
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, random_state=rng, format="csr")
    A.data = rng.uniform(0.5, 1.5, size=A.nnz)
    # zero out a few rows entirely to exercise empty rows
    if m > 8:
        dead = rng.choice(m, size=max(1, m // 16), replace=False)
        A = sp.csr_matrix(sp.diags(np.where(np.isin(np.arange(m), dead), 0.0, 1.0)) @ A)
        A.eliminate_zeros()
    x = rng.standard_normal(n)
    b, dn = add_noise(A @ x + 1e-3 * rng.standard_normal(m), noise, seed + 1)
    B = None
    if unmatched:
        At = A.T.tocsr()
        Bp = At.copy()
        Bp.data = Bp.data * (1.0 + 0.05 * rng.standard_normal(Bp.nnz))
        B = _as_int32_csr(Bp)
    return Problem(A=_as_int32_csr(A), B=B, b=b, x_true=x, noise_norm=dn, name="random")


def transpose_mismatch(A: sp.csr_matrix, B: sp.csr_matrix, seed: int = 0) -> float:
    """|y^T A x - x^T B y| for unit random x (n) and y (m) (paper, Sec. 3.2 CT test)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.shape[1])
    y = rng.standard_normal(A.shape[0])
    x /= np.linalg.norm(x)
    y /= np.linalg.norm(y)
    return float(abs(y @ (A @ x) - x @ (B @ y)))
