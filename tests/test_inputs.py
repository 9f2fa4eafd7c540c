"""Synthetic input generator: determinism and geometry sanity."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2605_22281_amd import inputs


def test_siddon_row_sums_are_chord_lengths():
    N, na, nd = 32, 12, 46
    A = inputs.siddon_matrix(N, na, nd)
    assert A.shape == (na * nd, N * N)
    theta = np.arange(na) * math.pi / na
    t = np.arange(nd) - (nd - 1) / 2
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(na, nd)
    half = N / 2
    for a in range(na):
        c, s = math.cos(theta[a]), math.sin(theta[a])
        for d in range(nd):
            # chord of the line {p . u = t} through the square [-half, half]^2
            vx, vy = -s, c
            ox, oy = t[d] * c, t[d] * s
            lo, hi = -1e9, 1e9
            for o, v in ((ox, vx), (oy, vy)):
                if abs(v) > 1e-15:
                    l1, l2 = (-half - o) / v, (half - o) / v
                    lo, hi = max(lo, min(l1, l2)), min(hi, max(l1, l2))
                elif abs(o) > half:
                    lo, hi = 0, 0
            chord = max(0.0, hi - lo)
            if abs(abs(t[d]) - half) > 1e-9:       # rays on the boundary edge are dropped
                assert abs(rs[a, d] - chord) < 1e-9, (a, d)


def test_siddon_entries_valid_and_sorted():
    A = inputs.siddon_matrix(24, 10, 35)
    assert A.indptr.dtype == np.int32 and A.indices.dtype == np.int32
    assert np.all(A.data > 0) and np.all(A.data <= math.sqrt(2) + 1e-12)
    for r in range(A.shape[0]):
        cols = A.indices[A.indptr[r]:A.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
    # every pixel is seen from every angle roughly once (column sums ~ number of angles)
    cs = np.asarray(A.sum(axis=0)).ravel()
    assert abs(cs.mean() - 10) < 0.5


def test_pixel_driven_backprojector_weights():
    N, na, nd = 32, 12, 46
    B = inputs.pixel_driven_backprojector(N, na, nd)
    assert B.shape == (N * N, na * nd)
    # interior pixels: the two interpolation weights of each angle sum to 1
    rs = np.asarray(B.sum(axis=1)).ravel()
    assert np.allclose(rs, na)
    A = inputs.siddon_matrix(N, na, nd)
    mm = inputs.transpose_mismatch(A, B)
    assert 1e-4 < mm < 0.2                      # unmatched, but close to A^T


def test_workload_sizes_and_determinism():
    P1 = inputs.workload("ct64")
    P2 = inputs.workload("ct64")
    assert P1.A.shape == (8190, 4096)
    assert abs(P1.A.nnz - 4.70e5) < 0.02e5
    assert np.array_equal(P1.b, P2.b) and np.array_equal(P1.x_true, P2.x_true)
    e = P1.b - P1.A @ P1.x_true
    assert abs(np.linalg.norm(e) - P1.noise_norm) < 1e-12 * P1.noise_norm
    assert abs(P1.noise_norm / np.linalg.norm(P1.A @ P1.x_true) - 0.01) < 1e-12


def test_phantoms():
    x = inputs.ellipse_phantom(64, seed=3)
    assert x.shape == (4096,) and x.min() >= 0 and x.max() > 0.2
    xs = inputs.sparse_phantom(64, seed=3)
    assert (xs != 0).sum() == round(0.02 * 4096)
    assert np.array_equal(xs, inputs.sparse_phantom(64, seed=3))


def test_batch_instances_uneven():
    insts = inputs.batch_instances(count=6, sides=(16, 24, 32), seed=4)
    sides = {p.N for p in insts}
    assert len(insts) == 6 and len(sides) >= 2
    for p in insts:
        na, nd = inputs.geometry_for_side(p.N)
        assert p.A.shape == (na * nd, p.N * p.N)
        lvl = p.noise_norm / np.linalg.norm(p.A @ p.x_true)
        assert 0.005 <= lvl <= 0.03
    # a selection builds the same instances as the whole batch
    drawn = inputs.batch_instance_sides(count=6, sides=(16, 24, 32), seed=4)
    assert [d[0] for d in drawn] == [p.N for p in insts]
    sub = inputs.batch_instances(count=6, sides=(16, 24, 32), seed=4, select=[4, 1])
    for q, i in zip(sub, (4, 1)):
        assert q.N == insts[i].N and np.array_equal(q.b, insts[i].b)
        assert np.array_equal(q.x_true, insts[i].x_true)


def test_random_sparse_problem_has_empty_rows():
    P = inputs.random_sparse_problem(100, 40, 0.1, seed=1, unmatched=True)
    lens = np.diff(P.A.indptr)
    assert (lens == 0).any()
    assert sp.issparse(P.B) and P.B.shape == (40, 100)


def test_tile_order_is_a_permutation_grouping_blocks():
    for N, T in ((8, 4), (10, 4), (24, 4), (16, 8)):
        perm = inputs.tile_order(N, T)
        assert perm.dtype == np.int32 and sorted(perm.tolist()) == list(range(N * N))
        # the pixels of one full block occupy T*T consecutive positions
        r0, c0 = T, 0
        block = [(r0 + i) * N + c0 + j for i in range(T) for j in range(T)]
        pos = np.sort(perm[block])
        assert pos[-1] - pos[0] == T * T - 1
    # renumbering the columns of a projector leaves each row's dot product unchanged
    P = inputs.small_ct(12, 10)
    perm = inputs.tile_order(12, 4)
    x = np.random.default_rng(0).standard_normal(P.n)
    xp = np.empty_like(x)
    xp[perm] = x
    Ap = sp.csr_matrix((P.A.data, perm[P.A.indices], P.A.indptr), shape=P.A.shape)
    assert np.allclose(Ap @ xp, P.A @ x, rtol=1e-14, atol=1e-14)


def test_deblur_operator():
    P = inputs.workload("deblur64")
    N = 64
    K = inputs.gaussian_blur_matrix(N, 0.25)
    # unit sum away from the boundary, symmetric, separable 5 x 5 stencil
    rs = np.asarray(K.sum(axis=1)).ravel().reshape(N, N)
    np.testing.assert_allclose(rs[2:-2, 2:-2], 1.0, rtol=1e-14)
    assert abs(K - K.T).max() < 1e-16 and K.getnnz(axis=1).max() == 25
    w = np.exp(-1.0 / 0.5)
    assert K[N * 10 + 10, N * 10 + 11] / K[N * 10 + 10, N * 10 + 10] == pytest.approx(w, rel=1e-13)
    assert P.m == round(0.7 * N * N) and P.n == N * N
    e = P.b - P.A @ P.x_true
    assert np.linalg.norm(e) == pytest.approx(0.05 * np.linalg.norm(P.A @ P.x_true), rel=1e-12)
    s = np.linalg.svd(P.x_true.reshape(N, N), compute_uv=False)
    assert s[10] < 0.05 * s[0]                 # quickly decaying spectrum
