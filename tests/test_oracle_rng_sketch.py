"""Pins of the oracle's random generator and sketching operators.

Philox4x64-10 is pinned to the published Random123 known-answer vectors and to
numpy's independent implementation; the sketches are pinned to their defining
properties (paper Sec. 2.7: the families; the embedding property of Sec. 2.3,
eq. (sketchProp)).
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import philox, sketches

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert list(philox.block(ctr, key)) == out
    got = philox.blocks(*[np.array([c], dtype=np.uint64) for c in ctr], key)
    assert [int(g[0]) for g in got] == out


def _numpy_block(ctr, key):
    # numpy.random.Philox increments its 256-bit counter before each block
    c = (sum(int(v) << (64 * i) for i, v in enumerate(ctr)) - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & philox.MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=words, key=np.array(key, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def test_philox_matches_numpy_bitgenerator():
    rng = np.random.default_rng(5)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] = int(rng.integers(0, 1 << 20))
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert list(philox.block(ctr, key)) == _numpy_block(ctr, key)


def test_philox_vectorised_equals_scalar():
    key = (123456789, 42 + (3 << 32))
    c0 = np.arange(0, 300, dtype=np.uint64)
    got = philox.blocks(c0, np.uint64(7), np.uint64(0), np.uint64(0), key)
    for i in range(300):
        assert tuple(int(g[i]) for g in got) == philox.block((i, 7, 0, 0), key)


def test_mulhi64_range():
    for n in (1, 2, 7, 65536, 2**31 - 1):
        assert philox.mulhi64(0, n) == 0
        assert philox.mulhi64(philox.MASK64, n) == n - 1


@pytest.mark.parametrize("d,s,zeta", [(37, 11, 3), (200, 50, 8), (64, 8, 8), (10, 5, 1)])
def test_sparse_sign_vectorised_equals_loop(d, s, zeta):
    r1, g1 = sketches.sparse_sign_codes_loop(d, s, zeta, seed=99)
    r2, g2 = sketches.sparse_sign_codes(d, s, zeta, seed=99)
    assert np.array_equal(r1, r2) and np.array_equal(g1, g2)


def test_sparse_sign_structure():
    d, s, zeta = 500, 40, 8
    S = sketches.SparseSign(d, s, zeta, seed=7)
    M = S.matrix()
    nnz_per_col = (M != 0).sum(axis=0)
    assert np.all(nnz_per_col == zeta)                   # zeta distinct rows per column
    assert np.allclose(np.abs(M[M != 0]), 1 / math.sqrt(zeta))
    assert np.allclose(np.linalg.norm(M, axis=0), 1.0)   # unit columns
    # rows roughly uniformly used and both signs present
    assert (M > 0).sum() > 0.4 * d * zeta and (M < 0).sum() > 0.4 * d * zeta
    counts = (M != 0).sum(axis=1)
    assert counts.min() > 0.5 * d * zeta / s


def test_countsketch_is_zeta_one():
    S = sketches.make("countsketch", 64, 9, seed=3)
    M = S.matrix()
    assert np.all((M != 0).sum(axis=0) == 1)
    assert set(np.unique(M[M != 0])) <= {-1.0, 1.0}


@pytest.mark.parametrize("N", [1, 2, 8, 64, 1024])
def test_fwht_equals_sylvester_hadamard(N):
    x = np.random.default_rng(N).standard_normal(N)
    assert np.allclose(sketches.fwht(x), sla.hadamard(N) @ x, rtol=0, atol=1e-12 * N)


def test_srht_is_scaled_row_orthonormal():
    # with d = N (no padding) H_N D is orthogonal, so S S^T = (N / s) R R^T = (N / s) I_s
    d, s = 256, 40
    S = sketches.SRHT(d, s, seed=11)
    M = S.matrix()
    assert np.allclose(M @ M.T, (d / s) * np.eye(s), atol=1e-12)
    assert len(set(S.rows.tolist())) == s
    assert set(np.unique(S.D)) <= {-1.0, 1.0}
    H = sla.hadamard(d) / math.sqrt(d)
    explicit = math.sqrt(d / s) * (H @ np.diag(S.D))[S.rows]
    assert np.allclose(M, explicit, atol=1e-13)


def test_srht_padding():
    d, s = 100, 30
    S = sketches.SRHT(d, s, seed=2)
    assert S.N == 128
    v = np.random.default_rng(0).standard_normal(d)
    u = np.concatenate([v, np.zeros(28)])
    H = sla.hadamard(128) / math.sqrt(128)
    assert np.allclose(S.apply(v), math.sqrt(128 / s) * (H @ (S.D * u))[S.rows], atol=1e-13)


def test_srht_rows_are_fisher_yates_prefix():
    # the selected rows are the first s entries of a shuffle of [0, N): distinct, in range,
    # and selecting s = N gives a permutation
    N = 64
    r = sketches.srht_rows(N, N, seed=5)
    assert sorted(r.tolist()) == list(range(N))
    assert np.array_equal(sketches.srht_rows(N, 10, seed=5), r[:10])


@pytest.mark.parametrize("kind", ["sparse_sign", "srht", "gaussian"])
def test_subspace_embedding_distortion(kind):
    # eq. (sketchProp): (1-eps)||v|| <= ||S v|| <= (1+eps)||v|| on a (k+1)-dim subspace
    m, k = 4096, 20
    s = 8 * (k + 1)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((m, k + 1)))
    S = sketches.make(kind, m, s, seed=17, zeta=8)
    SQ = np.stack([S.apply(Q[:, j]) for j in range(k + 1)], axis=1)
    sv = np.linalg.svd(SQ, compute_uv=False)
    assert sv.max() < 1.5 and sv.min() > 0.5
