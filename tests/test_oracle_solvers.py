"""Pins of the step-by-step sFLSQR / sFLSMR oracle against what the paper and
the mathematics fix.  Each test names the passage it checks.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import dense, fgk, sketches
from paper_2605_22281_amd import inputs


def well_conditioned(m, n, cond, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = np.geomspace(1.0, 1.0 / cond, n)
    A = (U * sig) @ V.T
    b = rng.standard_normal(m)
    return A, b


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --- Sec. 2.1-2.2: tau = I and B = A^T reduce FGK to Golub-Kahan, so the sketch-free
# variants are LSQR and LSMR (eq. (xlsqr), eq. (xlsmr)).

@pytest.mark.parametrize("ell", [1, 2, 5])
def test_sflsqr_identity_sketch_is_lsqr(ell):
    # small condition number and few steps: both short recurrences stay orthogonal
    A, b = well_conditioned(60, 30, 10.0, seed=1)
    r = fgk.sketched_flexible(A, b, sketches.Identity(60), method="sflsqr", maxit=10, ell=ell)
    for k in range(1, 11):
        xl = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert rel(r.X[:, k - 1], xl) < 1e-10, k


@pytest.mark.parametrize("ell", [1, 2])
def test_sflsmr_identity_sketch_is_lsmr(ell):
    A, b = well_conditioned(60, 30, 10.0, seed=2)
    r = fgk.sketched_flexible(A, b, sketches.Identity(30), method="sflsmr", maxit=10, ell=ell)
    for k in range(1, 11):
        xm = spla.lsmr(A, b, atol=0, btol=0, conlim=0, maxiter=k)[0]
        assert rel(r.X[:, k - 1], xm) < 1e-10, k


# --- Sec. 2.2 vs 2.3: with S = I and a window covering all previous vectors, the
# sketched solvers coincide with FLSQR / FLSMR written from eq. (FLSQR) and the FLSMR
# formula (which rely on the orthonormality of W and P).  ell = maxit - 1 is the
# smallest window that stays complete, so a window one too short fails here.

@pytest.mark.parametrize("tau", ["identity", "reweight_l1"])
def test_full_window_equals_flsqr(tau):
    P = inputs.random_sparse_problem(80, 40, 0.2, seed=3, unmatched=True)
    maxit = 12
    r = fgk.sketched_flexible(P.A, P.b, sketches.Identity(80), method="sflsqr", B=P.B,
                              maxit=maxit, ell=maxit - 1, tau=tau, eps=0.3)
    f = fgk.flexible_full(P.A, P.b, method="flsqr", B=P.B, maxit=maxit, tau=tau, eps=0.3)
    for k in range(maxit):
        assert rel(r.X[:, k], f.X[:, k]) < 1e-9, k
        assert abs(r.rho[k] - f.rho[k]) <= 1e-9 * f.rho[k]


@pytest.mark.parametrize("tau", ["identity", "reweight_l1"])
def test_full_window_equals_flsmr(tau):
    P = inputs.random_sparse_problem(80, 40, 0.2, seed=4, unmatched=True)
    maxit = 12
    r = fgk.sketched_flexible(P.A, P.b, sketches.Identity(40), method="sflsmr", B=P.B,
                              maxit=maxit, ell=maxit - 1, tau=tau, eps=0.3)
    f = fgk.flexible_full(P.A, P.b, method="flsmr", B=P.B, maxit=maxit, tau=tau, eps=0.3)
    for k in range(maxit):
        assert rel(r.X[:, k], f.X[:, k]) < 1e-9, k


def test_full_window_w_and_p_orthonormal():
    P = inputs.random_sparse_problem(80, 40, 0.2, seed=5, unmatched=True)
    r = fgk.sketched_flexible(P.A, P.b, sketches.Identity(80), B=P.B, maxit=10, ell=20,
                              tau="reweight_l1", eps=0.2)
    assert np.abs(r.W.T @ r.W - np.eye(11)).max() < 1e-12
    assert np.abs(r.P.T @ r.P - np.eye(10)).max() < 1e-12


# --- ell = 0: the z-side window is empty, so p_k = B w_k / ||B w_k||, and w_{k+1} is
# A z_k with only its w_k component removed (closed form of the loops of Alg. 1).

def test_window_zero_closed_form():
    P = inputs.random_sparse_problem(50, 30, 0.3, seed=6, unmatched=True)
    S = sketches.make("sparse_sign", 50, 25, seed=1, zeta=3)
    r = fgk.sketched_flexible(P.A, P.b, S, B=P.B, maxit=6, ell=0, tau="reweight_l1", eps=0.5)
    for k in range(6):
        Bw = P.B @ r.W[:, k]
        assert rel(r.P[:, k], Bw / np.linalg.norm(Bw)) < 1e-13
        Az = P.A @ r.Z[:, k]
        v = Az - (r.W[:, k] @ Az) * r.W[:, k]
        assert rel(r.W[:, k + 1], v / np.linalg.norm(v)) < 1e-12


# --- eq. (FGK): A Z_k = W_{k+1} H_{k+1,k} and B W_k = P_k T_k hold to rounding, with H
# and T banded (entries older than the window are zero).

@pytest.mark.parametrize("method", ["sflsqr", "sflsmr"])
def test_recurrence_invariants_and_band(method):
    P = inputs.small_ct(16, 12, unmatched=True)
    d = P.m if method == "sflsqr" else P.n
    S = sketches.make("sparse_sign", d, 60, seed=2, zeta=4)
    ell, k = 2, 25
    r = fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=k, ell=ell,
                              tau="reweight_l1", eps=1e-2)
    Anorm = sp.linalg.norm(P.A)
    assert np.linalg.norm(P.A @ r.Z - r.W @ r.H) <= 1e-13 * Anorm * math.sqrt(k)
    assert np.linalg.norm(P.B @ r.W[:, :k] - r.P @ r.T) <= 1e-13 * sp.linalg.norm(P.B) * math.sqrt(k)
    for j in range(k):
        assert np.all(r.H[: max(0, j - ell), j] == 0) and np.all(r.H[j + 2:, j] == 0)
        assert np.all(r.T[: max(0, j - ell), j] == 0) and np.all(r.T[j + 1:, j] == 0)


# --- eq. (sFLSQR) / eq. (sFLSMR): the step-wise solution equals the definitional dense
# form on the same basis, with an explicit sketch matrix.

@pytest.mark.parametrize("method,kind", [("sflsqr", "sparse_sign"), ("sflsqr", "srht"),
                                         ("sflsmr", "sparse_sign"), ("sflsmr", "srht"),
                                         ("sflsqr", "gaussian")])
def test_stepwise_equals_definition(method, kind):
    P = inputs.random_sparse_problem(64, 48, 0.25, seed=8, unmatched=True)
    d = 64 if method == "sflsqr" else 48
    S = sketches.make(kind, d, 30, seed=5, zeta=4)
    r = fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=12, ell=2,
                              tau="reweight_l1", eps=0.1)
    Sm = S.matrix()
    for k in range(1, 13):
        Zk = r.Z[:, :k]
        if method == "sflsqr":
            xd = dense.sflsqr_from_basis(P.A, P.b, Sm, Zk)
        else:
            xd = dense.sflsmr_from_basis(P.A, P.b, Sm, Zk, B=P.B)
        assert rel(r.X[:, k - 1], xd) < 1e-9, k


# --- n steps on a well-conditioned square problem span R^n: the result is the dense
# least-squares solution of the sketched problem (and of the plain one when S = I).

def test_n_steps_reach_dense_lstsq():
    A, b = well_conditioned(40, 12, 10.0, seed=9)
    S = sketches.make("sparse_sign", 40, 30, seed=3, zeta=4)
    r = fgk.sketched_flexible(A, b, S, method="sflsqr", maxit=12, ell=2)
    Sm = S.matrix()
    xs = np.linalg.lstsq(Sm @ A, Sm @ b, rcond=None)[0]
    assert rel(r.x, xs) < 1e-10
    r2 = fgk.sketched_flexible(A, b, sketches.Identity(40), method="sflsqr", maxit=12, ell=2)
    assert rel(r2.x, np.linalg.lstsq(A, b, rcond=None)[0]) < 1e-10
    # sFLSMR: with s = n = 16 the SRHT is a scaled orthogonal matrix, so the sketched
    # normal equations are the normal equations
    A16, b16 = well_conditioned(40, 16, 10.0, seed=19)
    r3 = fgk.sketched_flexible(A16, b16, sketches.make("srht", 16, 16, seed=1), method="sflsmr",
                               maxit=16, ell=2)
    assert rel(r3.x, np.linalg.lstsq(A16, b16, rcond=None)[0]) < 1e-9


# --- Remark after Alg. 2: sFLSMR with sketch S equals sFLSQR with sketch S A^T (here S B).

def test_remark_sflsmr_is_sflsqr_with_sketch_SB():
    P = inputs.random_sparse_problem(70, 50, 0.2, seed=10, unmatched=True)
    S = sketches.make("srht", 50, 40, seed=4)
    # 9 steps: the sketched matrices stay well conditioned (cond < 1e7), beyond which the
    # two algebraically equal forms differ by eps * cond
    r1 = fgk.sketched_flexible(P.A, P.b, S, method="sflsmr", B=P.B, maxit=9, ell=2)
    SB = sketches.Dense(S.matrix() @ P.B.toarray())
    r2 = fgk.sketched_flexible(P.A, P.b, SB, method="sflsqr", B=P.B, maxit=9, ell=2)
    for k in range(9):
        assert rel(r1.X[:, k], r2.X[:, k]) < 1e-9, k
        assert abs(r1.rho[k] - r2.rho[k]) <= 1e-8 * r2.rho[k]


# --- Remark (spectral decay): if rank(A) = k, after k steps r^sFLSMR equals r^opt.

def test_rank_k_sflsmr_is_optimal():
    rng = np.random.default_rng(12)
    k = 6
    A = rng.standard_normal((50, k)) @ rng.standard_normal((k, 30))
    b = rng.standard_normal(50)
    S = sketches.make("gaussian", 30, 20, seed=6)
    r = fgk.sketched_flexible(A, b, S, method="sflsmr", maxit=k, ell=2)
    r_opt = dense.optimal_residual(A, b, r.Z)
    assert abs(r.res_true[-1] - r_opt) <= 1e-9 * r_opt
    rq = fgk.sketched_flexible(A, b, sketches.make("gaussian", 50, 20, seed=6), method="sflsqr",
                               maxit=k, ell=2)
    assert rq.res_true[-1] > r_opt * (1 + 1e-6)        # sFLSQR is not optimal in general


# --- Theorem 1: both residual bounds hold at every step.

@pytest.mark.parametrize("kind", ["gaussian", "sparse_sign"])
def test_theorem1_bounds(kind):
    P = inputs.random_sparse_problem(90, 40, 0.2, seed=13)
    for method in ("sflsqr", "sflsmr"):
        d = 90 if method == "sflsqr" else 40
        S = sketches.make(kind, d, 31, seed=8, zeta=4)
        r = fgk.sketched_flexible(P.A, P.b, S, method=method, maxit=14, ell=2)
        Sm = S.matrix()
        for k in range(1, 15):
            Zk = r.Z[:, :k]
            if method == "sflsqr":
                r_opt, bound, _ = dense.theorem1_bounds(P.A, P.b, Zk, S_m=Sm)
            else:
                r_opt, _, bound = dense.theorem1_bounds(P.A, P.b, Zk, S_n=Sm)
            assert r_opt <= r.res_true[k - 1] * (1 + 1e-10)
            assert r.res_true[k - 1] <= bound * (1 + 1e-10), (method, k)


# --- Corollary 1 (with numerator k, see the oracle's note): Gaussian S independent of
# the basis gives E[(r^sFLSQR)^2] = (r^opt)^2 (1 + k / (s - k - 1)).

def test_corollary1_expectation_monte_carlo():
    rng = np.random.default_rng(14)
    m, k, s, trials = 200, 8, 22, 4000
    AZ = rng.standard_normal((m, k))
    b = rng.standard_normal(m)
    y_opt = np.linalg.lstsq(AZ, b, rcond=None)[0]
    r_opt2 = float(np.sum((AZ @ y_opt - b) ** 2))
    vals = np.empty(trials)
    for t in range(trials):
        G = rng.standard_normal((s, m))
        y = np.linalg.lstsq(G @ AZ, G @ b, rcond=None)[0]
        vals[t] = np.sum((AZ @ y - b) ** 2)
    mean = vals.mean() / r_opt2
    sem = vals.std() / math.sqrt(trials) / r_opt2
    assert abs(mean - dense.corollary1_factor(k, s)) < 4 * sem
    printed = 1 + s / (s - k - 1)
    assert abs(mean - printed) > 10 * sem                # the printed numerator s is refuted


# --- eq. (discrP) / Alg. 1 stop test: the run stops at the first k with
# rho_k < tol ||S b||, and x is that iterate.

def test_discrepancy_stop_is_first_crossing():
    P = inputs.small_ct(24, 18, noise=0.05)
    S = sketches.make("sparse_sign", P.m, 80, seed=9, zeta=8)
    full = fgk.sketched_flexible(P.A, P.b, S, maxit=30, ell=2)
    tol = fgk.discrepancy_tol(1.01, P.noise_norm, full.beta)
    k_expect = int(np.argmax(full.rho < tol * full.rhs_norm)) + 1
    assert full.rho[k_expect - 1] < tol * full.rhs_norm
    r = fgk.sketched_flexible(P.A, P.b, S, maxit=30, ell=2, tol=tol)
    assert r.stopped and r.k == k_expect
    assert np.array_equal(r.x, full.X[:, k_expect - 1])


# --- A = I: the first step reaches b exactly and h_{2,1} = 0 (happy breakdown).

def test_happy_breakdown_identity_matrix():
    n = 20
    b = np.random.default_rng(15).standard_normal(n)
    S = sketches.make("sparse_sign", n, 10, seed=1, zeta=2)
    r = fgk.sketched_flexible(sp.identity(n, format="csr"), b, S, maxit=5, ell=2)
    assert r.breakdown and r.k == 1
    assert rel(r.x, b) < 1e-14


# --- Sec. 2.3 note: tau(v) = v makes sFLSQR 'sLSQR'; a reweighting with huge eps is a
# constant diagonal, which only rescales the basis: same iterates as tau = I.

def test_reweight_with_huge_eps_is_identity():
    P = inputs.small_ct(16, 12)
    S = sketches.make("sparse_sign", P.m, 40, seed=2, zeta=4)
    r1 = fgk.sketched_flexible(P.A, P.b, S, maxit=10, ell=2, tau="identity")
    r2 = fgk.sketched_flexible(P.A, P.b, S, maxit=10, ell=2, tau="reweight_l1", eps=1e8)
    for k in range(10):
        assert rel(r2.X[:, k], r1.X[:, k]) < 1e-10


def test_reweight_changes_iterates():
    P = inputs.small_ct(16, 12, phantom="sparse")
    S = sketches.make("sparse_sign", P.m, 40, seed=2, zeta=4)
    r1 = fgk.sketched_flexible(P.A, P.b, S, maxit=10, ell=2, tau="identity")
    r2 = fgk.sketched_flexible(P.A, P.b, S, maxit=10, ell=2, tau="reweight_l1", eps=1e-3)
    assert rel(r2.X[:, 9], r1.X[:, 9]) > 1e-3


# --- Sec. 2.4 synthetic experiment (weak pin): with Gaussian S, s = 2 maxit + 1, the
# final sLSQR residual is larger than LSQR's (the paper reports about +30%); sLSMR
# tracks LSQR more closely.

def test_artificial_experiment_residual_excess():
    maxit = 40
    for noise in (0.01, 0.10):
        P = inputs.artificial_problem(noise=noise, seed=16)
        A = P.A.toarray()
        xl = spla.lsqr(A, P.b, atol=0, btol=0, conlim=0, iter_lim=maxit)[0]
        r_lsqr = np.linalg.norm(A @ xl - P.b)
        q = fgk.sketched_flexible(A, P.b, sketches.make("gaussian", A.shape[0], 2 * maxit + 1, seed=1),
                                  method="sflsqr", maxit=maxit, ell=2)
        mr = fgk.sketched_flexible(A, P.b, sketches.make("gaussian", A.shape[1], 2 * maxit + 1, seed=1),
                                   method="sflsmr", maxit=maxit, ell=2)
        excess_q = q.res_true[-1] / r_lsqr - 1
        excess_m = mr.res_true[-1] / r_lsqr - 1
        assert 0.05 < excess_q < 1.0, (noise, excess_q)
        assert excess_m < excess_q


# --- Rounding sensitivity (property of the method, not of one implementation): two
# summation orders of the same products agree to ~1e-14 while the basis is still
# well conditioned; with tau = I on a CT problem the short-window basis loses rank
# after ~20 steps and the two runs separate; the l1 reweighting stays reproducible.

def _two_orders(P, tau, maxit):
    S = sketches.make("sparse_sign", P.m, 200, seed=3001, zeta=8)
    r1 = fgk.sketched_flexible(P.A, P.b, S, maxit=maxit, ell=2, tau=tau)
    rng = np.random.default_rng(0)
    pc = rng.permutation(P.n)
    pr = rng.permutation(P.m)
    Ap = P.A[:, pc].tocsr()
    Ap.sort_indices()                      # sum each row in the permuted column order
    Bp = P.A.T.tocsr()[:, pr].tocsr()
    Bp.sort_indices()
    r2 = fgk.sketched_flexible(lambda v: Ap @ v[pc], P.b, S, B=lambda v: Bp @ v[pr], maxit=maxit,
                               ell=2, tau=tau, m=P.m, n=P.n)
    return np.array([rel(r2.X[:, k], r1.X[:, k]) for k in range(maxit)])


def test_rounding_sensitivity_horizon():
    P = inputs.workload("ct64")
    dev_id = _two_orders(P, "identity", 40)
    assert dev_id[:12].max() < 1e-12               # well conditioned: reproducible
    assert dev_id[30:].max() > 1e-6                # lost rank: not determined by the arithmetic
    dev_rw = _two_orders(P, "reweight_l1", 40)
    assert dev_rw.max() < 1e-12
