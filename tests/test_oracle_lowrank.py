"""Pins of the low-rank truncation oracle (oracle/lowrank.py) against closed
forms, the Eckart-Young theorem (through a symmetric eigensolver, not the SVD),
invariances of eq. (def:lowr-trc), the exact-recovery property and error bound
of the randomized SVD (Halko-Martinsson-Tropp), and statistics of its Gaussian
test matrix."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as st

from oracle import fgk, lowrank, philox, sketches

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _spectrum_matrix(nr, nc, sig, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((nr, len(sig))))
    V, _ = np.linalg.qr(rng.standard_normal((nc, len(sig))))
    return (U * sig) @ V.T


def test_permuted_diagonal_closed_form():
    # C = P diag(d) Q^T (P, Q permutations): tau_r keeps the r entries of largest |d|
    rng = np.random.default_rng(1)
    n = 12
    d = rng.permutation(np.arange(1, n + 1, dtype=float)) * rng.choice([-1.0, 1.0], n)
    pr, pc = rng.permutation(n), rng.permutation(n)
    C = np.zeros((n, n))
    C[pr, pc] = d
    for r in (1, 4, 11):
        keep = np.abs(d) > n - r
        E = np.zeros((n, n))
        E[pr[keep], pc[keep]] = d[keep]
        got = lowrank.truncate(C.ravel(), n, n, r).reshape(n, n)
        np.testing.assert_allclose(got, E, atol=1e-13)


@pytest.mark.parametrize("nr,nc,r", [(16, 16, 3), (20, 12, 5), (9, 30, 8)])
def test_eckart_young_through_eigvalsh(nr, nc, r):
    rng = np.random.default_rng(nr * 100 + nc)
    C = rng.standard_normal((nr, nc))
    Cr = lowrank.truncate(C.ravel(), nr, nc, r).reshape(nr, nc)
    lam = np.sort(sla.eigvalsh(C.T @ C if nc <= nr else C @ C.T))[::-1]
    tail = float(np.sum(lam[r:]))
    err2 = float(np.linalg.norm(C - Cr) ** 2)
    assert abs(err2 - tail) <= 1e-10 * float(np.sum(lam))
    assert np.linalg.matrix_rank(Cr, tol=1e-10 * np.abs(Cr).max()) == r
    # no rank-r matrix does better
    for t in range(20):
        B = rng.standard_normal((nr, r)) @ rng.standard_normal((r, nc))
        B = Cr + 1e-2 * B
        Bt = lowrank.truncate(B.ravel(), nr, nc, r).reshape(nr, nc)
        assert np.linalg.norm(C - Bt) >= np.linalg.norm(C - Cr) * (1 - 1e-12)


def test_invariances():
    rng = np.random.default_rng(3)
    nr, nc, r = 14, 10, 4
    sig = np.array([9.0, 7.0, 5.0, 4.0, 2.0, 1.5, 1.0, 0.5, 0.2, 0.1])
    C = _spectrum_matrix(nr, nc, sig, 4)
    Cr = lowrank.truncate(C.ravel(), nr, nc, r).reshape(nr, nc)
    # orthogonal invariance: tau_r(U C V^T) = U tau_r(C) V^T
    U, _ = np.linalg.qr(rng.standard_normal((nr, nr)))
    V, _ = np.linalg.qr(rng.standard_normal((nc, nc)))
    got = lowrank.truncate((U @ C @ V.T).ravel(), nr, nc, r).reshape(nr, nc)
    np.testing.assert_allclose(got, U @ Cr @ V.T, atol=1e-12)
    # the order of vectorisation does not matter: (C^T)_r = (C_r)^T
    gt = lowrank.truncate(C.T.ravel(), nc, nr, r).reshape(nc, nr)
    np.testing.assert_allclose(gt.T, Cr, atol=1e-12)
    # idempotent and positively / negatively homogeneous
    np.testing.assert_allclose(lowrank.truncate(Cr.ravel(), nr, nc, r), Cr.ravel(), atol=1e-12)
    np.testing.assert_allclose(lowrank.truncate(-3.7 * C.ravel(), nr, nc, r), -3.7 * Cr.ravel(),
                               atol=1e-12)
    # the truncation keeps exactly the leading singular triplets
    np.testing.assert_allclose(np.linalg.svd(Cr, compute_uv=False)[:r], sig[:r], rtol=1e-12)


def test_degenerate_cases():
    c = np.random.default_rng(5).standard_normal(6 * 8)
    np.testing.assert_array_equal(lowrank.truncate(c, 6, 8, 6), c)
    np.testing.assert_array_equal(lowrank.truncate(c, 6, 8, 9), c)
    assert not np.any(lowrank.truncate(np.zeros(48), 6, 8, 2))
    np.testing.assert_array_equal(lowrank.randomized_truncate(c, 6, 8, 6), c)
    with pytest.raises(ValueError):
        lowrank.truncate(c, 7, 8, 2)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_randomized_recovers_exact_truncation_of_low_rank_matrix(q):
    # rank(C) <= l: the range finder captures range(C) (HMT Sec. 1.3 / Thm 9.1),
    # so the randomized truncation equals the exact one
    nr, nc, r, p = 40, 30, 5, 10
    sig = np.array([10.0, 8.0, 6.0, 5.0, 4.0, 2.0, 1.0, 0.5, 0.25, 0.1, 0.05, 0.01])
    C = _spectrum_matrix(nr, nc, sig, 6)
    ex = lowrank.truncate(C.ravel(), nr, nc, r)
    rn = lowrank.randomized_truncate(C.ravel(), nr, nc, r, p=p, q=q, seed=11, call=3)
    np.testing.assert_allclose(rn, ex, atol=1e-11 * np.abs(ex).max())


def test_randomized_converges_with_power_iterations():
    nr, nc, r = 60, 50, 4
    sig = 0.8 ** np.arange(50)
    C = _spectrum_matrix(nr, nc, sig, 7)
    ex = lowrank.truncate(C.ravel(), nr, nc, r)
    errs = [np.linalg.norm(lowrank.randomized_truncate(C.ravel(), nr, nc, r, p=2, q=q, seed=1)
                           - ex) for q in (0, 2, 8, 40)]
    assert errs[0] > errs[1] > errs[2] and errs[3] < 1e-10 * np.linalg.norm(ex)


def test_randomized_error_bound_in_expectation():
    # HMT Thm 10.5 (q = 0): E ||(I - Q Q^T) C||_F <= sqrt(1 + r / (p - 1)) tail_F,
    # and the rank-r truncation of Q Q^T C adds at most tail_F
    nr, nc, r, p = 80, 60, 6, 6
    sig = 1.0 / (1.0 + np.arange(60)) ** 1.2
    C = _spectrum_matrix(nr, nc, sig, 8)
    tail = math.sqrt(float(np.sum(sig[r:] ** 2)))
    errs = [np.linalg.norm(lowrank.randomized_truncate(C.ravel(), nr, nc, r, p=p, q=0, seed=2,
                                                        call=k) - C.ravel()) for k in range(1, 41)]
    bound = (1.0 + math.sqrt(1.0 + r / (p - 1))) * tail
    assert np.mean(errs) <= bound
    assert min(errs) >= tail * (1 - 1e-12)         # never beats Eckart-Young


def test_gaussian_test_matrix_statistics_and_layout():
    Om = lowrank.gaussian_test_matrix(1000, 50, seed=9, call=1)
    assert Om.shape == (1000, 50)
    v = Om.ravel()
    assert abs(v.mean()) < 0.02 and abs(v.var() - 1.0) < 0.03
    assert st.kstest(v, "norm").pvalue > 1e-3
    Om2 = lowrank.gaussian_test_matrix(1000, 50, seed=9, call=2)
    assert abs(np.corrcoef(Om.ravel(), Om2.ravel())[0, 1]) < 0.02
    assert abs(np.corrcoef(Om[:, 0], Om[:, 1])[0, 1]) < 0.1
    # entry e = j * nc + i from a scalar Philox block and Box-Muller
    key = (9, lowrank.STREAM_LOWRANK)
    for (i, j) in [(0, 0), (3, 0), (999, 7), (5, 49)]:
        e = j * 1000 + i
        w = philox.block((1, e >> 2, 0, 0), key)
        t = e & 3
        u1 = ((w[2 * (t // 2)] >> 11) + 0.5) * 2.0 ** -53
        u2 = (w[2 * (t // 2) + 1] >> 11) * 2.0 ** -53
        val = math.sqrt(-2 * math.log(u1)) * (math.cos if t % 2 == 0 else math.sin)(2 * math.pi * u2)
        assert Om[i, j] == pytest.approx(val, rel=1e-14, abs=1e-15)


def test_solver_with_full_rank_truncation_is_the_plain_solver():
    # r >= N makes tau_r the identity: FLSQR with it is FLSQR with tau = I, and
    # every z_k of a rank-r run has rank <= r and equals tau_r(p_k)
    rng = np.random.default_rng(12)
    N = 8
    A = rng.standard_normal((90, N * N))
    b = rng.standard_normal(90)
    full = fgk.flexible_full(A, b, maxit=10, tau=lowrank.Truncation(N, N, N))
    ident = fgk.flexible_full(A, b, maxit=10, tau="identity")
    np.testing.assert_allclose(full.X, ident.X, rtol=1e-12, atol=1e-14)
    S = sketches.SparseSign(90, 40, 1, 3)
    res = fgk.sketched_flexible(A, b, S, maxit=12, tau=lowrank.Truncation(N, N, 2))
    for k in range(res.k):
        zk = res.Z[:, k].reshape(N, N)
        assert np.linalg.svd(zk, compute_uv=False)[2] <= 1e-13 * np.linalg.norm(zk)
        np.testing.assert_allclose(res.Z[:, k], lowrank.truncate(res.P[:, k], N, N, 2), atol=1e-14)
    # eq. (FGK): A Z_k = W_{k+1} H_{k+1,k} holds for the truncated basis too
    k = res.k
    np.testing.assert_allclose(A @ res.Z, res.W[:, :k + 1] @ res.H, atol=1e-10)


def test_randomized_operator_draws_a_new_matrix_per_call():
    N = 10
    c = np.random.default_rng(13).standard_normal(N * N)
    t = lowrank.RandomizedTruncation(N, N, 3, p=2, q=0, seed=4)
    a, b2 = t(c, None, 1), t(c, None, 2)
    assert np.linalg.norm(a - b2) > 1e-6
    np.testing.assert_array_equal(a, t(c, None, 1))
