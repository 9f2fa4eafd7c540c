"""Low-rank flexible operators on the GPU (tau LOWRANK: truncated SVD to a
Ritz-residual tolerance; LOWRANK_RND: the randomized SVD) against the oracle:
the operator alone through sfk_tau_apply, then sFLSQR, sFLSMR and FLSQR with it
on the 64^2 deblurring problem, and properties that hold at any step.

Tolerance of the truncated-SVD variant: its Ritz residuals are at most
tol * theta_1 (tol = 1e-13), so the computed rank-r subspace is within
tol * sigma_1^2 / (sigma_r^2 - sigma_{r+1}^2) of the exact one; the test allows
20 sqrt(r) times that (plus 1e-12) relative to ||C_r||."""
import math

import numpy as np
import pytest

from oracle import fgk, lowrank, sketches
from paper_2605_22281_amd import inputs

from gpu_cases import gpu_run, pinned, rel, say

pytestmark = pytest.mark.gpu


def _ctx_for(nr, nc, tau, r, **kw):
    """A context whose unknowns form an nr x nc image (the operator is not used
    by sfk_tau_apply; a small random sparse problem carries it)."""
    import torch
    from paper_2605_22281_amd import sfk
    P = inputs.random_sparse_problem(nr * nc + 64, nr * nc, 0.002, seed=nr * 7 + nc)
    A = sfk.to_device_csr(P.A)
    b = torch.from_numpy(np.ascontiguousarray(P.b)).cuda()
    p = sfk.params("sflsqr", ell=2, maxit=20, sketch="sparse_sign", s=64, zeta=1, seed=21,
                   tau=tau, lr_rows=nr, lr_rank=r, **kw)
    return sfk.init(A, None, b, p), A, b


def _spectrum_matrix(nr, nc, sig, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((nr, len(sig))))
    V, _ = np.linalg.qr(rng.standard_normal((nc, len(sig))))
    return (U * sig) @ V.T


def _bound(C, r, tol=1e-13):
    s = np.linalg.svd(C, compute_uv=False)
    gap = s[r - 1] ** 2 - s[r] ** 2
    return 1e-12 + 20.0 * math.sqrt(r) * tol * s[0] ** 2 / gap


CASES = [
    ("decay64", 64, 64, 10, lambda: _spectrum_matrix(64, 64, 0.9 ** np.arange(64), 1)),
    ("gauss64", 64, 64, 8, lambda: np.random.default_rng(2).standard_normal((64, 64))),
    ("rect40x96", 40, 96, 6, lambda: np.random.default_rng(3).standard_normal((40, 96))
     + 5.0 * np.outer(np.linspace(1, 2, 40), np.cos(np.arange(96) / 9.0))),
    ("r30_of_128", 128, 128, 30, lambda: _spectrum_matrix(128, 128, 1.0 / (1.0 + np.arange(128)),
                                                          4)),
]


@pytest.mark.parametrize("name,nr,nc,r,make", CASES, ids=[c[0] for c in CASES])
def test_truncated_svd_operator_against_oracle(name, nr, nc, r, make):
    import torch
    from paper_2605_22281_amd import sfk
    say(f"case: lowrank operator {name} {nr}x{nc} r={r}")
    C = make()
    ctx, _, _ = _ctx_for(nr, nc, "lowrank", r)
    try:
        got = sfk.tau_apply(ctx, torch.from_numpy(C.ravel()).cuda(), call=1).cpu().numpy()
        st = sfk.tau_stats(ctx)
    finally:
        sfk.destroy(ctx)
    ref = lowrank.truncate(C.ravel(), nr, nc, r)
    err = rel(got, ref)
    bnd = _bound(C, r)
    say(f"{name}: rel err {err:.2e} (bound {bnd:.1e}), {st['iterations']} power iterations, "
        f"residual {st['resmax']:.1e}")
    assert st["converged"] and st["resmax"] <= 1e-13
    assert err <= bnd
    # the output has rank r
    sv = np.linalg.svd(got.reshape(nr, nc), compute_uv=False)
    assert sv[r] <= 1e-12 * sv[0]


@pytest.mark.parametrize("q", [0, 1, 2])
def test_randomized_operator_against_oracle(q):
    import torch
    from paper_2605_22281_amd import sfk
    nr, nc, r = 64, 64, 10
    C = _spectrum_matrix(nr, nc, 0.85 ** np.arange(64), 5)
    say(f"case: lowrank_rnd operator q={q}")
    ctx, _, _ = _ctx_for(nr, nc, "lowrank_rnd", r, lr_q=q)
    try:
        got = [sfk.tau_apply(ctx, torch.from_numpy(C.ravel()).cuda(), call=c).cpu().numpy()
               for c in (1, 2, 7)]
    finally:
        sfk.destroy(ctx)
    for c, g in zip((1, 2, 7), got):
        ref = lowrank.randomized_truncate(C.ravel(), nr, nc, r, p=10, q=q, seed=21, call=c)
        err = rel(g, ref)
        say(f"rnd q={q} call={c}: rel err {err:.2e}")
        assert err <= 1e-10
    if q == 0:
        assert rel(got[0], got[1]) > 1e-8       # a new test matrix per call


@pytest.mark.parametrize("tau", ["lowrank", "lowrank_rnd"])
def test_degenerate_inputs(tau):
    import torch
    from paper_2605_22281_amd import sfk
    nr, nc, r = 48, 48, 8
    low = _spectrum_matrix(nr, nc, np.array([5.0, 3.0, 2.0, 1.0, 0.5]), 6)   # rank 5 < r
    say(f"case: lowrank degenerate {tau}")
    ctx, _, _ = _ctx_for(nr, nc, tau, r)
    try:
        out = sfk.tau_apply(ctx, torch.from_numpy(low.ravel()).cuda()).cpu().numpy()
        zero = sfk.tau_apply(ctx, torch.zeros(nr * nc, dtype=torch.float64, device="cuda")).cpu().numpy()
        scaled = sfk.tau_apply(ctx, torch.from_numpy(-3.0 * low.ravel()).cuda()).cpu().numpy()
    finally:
        sfk.destroy(ctx)
    # rank below r: the truncation is the identity
    assert rel(out, low.ravel()) <= 1e-11
    assert not np.any(zero) and np.all(np.isfinite(zero))
    assert rel(scaled, -3.0 * out) <= 1e-11


def _oracle_tau(tau, N, r, q=1, seed=3001):
    if tau == "lowrank":
        return lowrank.Truncation(N, N, r)
    return lowrank.RandomizedTruncation(N, N, r, p=10, q=q, seed=seed)


def _oracle(P, method, tau_obj, K, s=101, seed=3001, permuted=False):
    """The oracle run; permuted: the same run with the products summed in
    another order (columns of A and B permuted and the vectors with them), a
    second correctly rounded result whose distance measures the method's
    sensitivity to rounding on this problem."""
    A, B = P.A, P.A.T.tocsr()
    kw = {}
    if permuted:
        rng = np.random.default_rng(0)
        pc, pr = rng.permutation(P.n), rng.permutation(P.m)
        Ap, Bp = A[:, pc].tocsr(), B[:, pr].tocsr()
        Ap.sort_indices()
        Bp.sort_indices()
        A, B = (lambda v: Ap @ v[pc]), (lambda v: Bp @ v[pr])
        kw = dict(m=P.m, n=P.n) if method not in ("flsqr", "flsmr") else {}
    if method in ("flsqr", "flsmr"):
        return fgk.flexible_full(A, P.b, method=method, B=B, maxit=K, tau=tau_obj)
    S = sketches.make("sparse_sign", P.m if method == "sflsqr" else P.n, s, seed, zeta=1)
    return fgk.sketched_flexible(A, P.b, S, method=method, B=B, maxit=K, tau=tau_obj, **kw)


@pytest.mark.parametrize("method,tau", [("sflsqr", "lowrank"), ("sflsmr", "lowrank"),
                                        ("flsqr", "lowrank"), ("sflsqr", "lowrank_rnd"),
                                        ("sflsmr", "lowrank_rnd")])
def test_solvers_with_lowrank_tau_deblur64(method, tau):
    """64^2 Gaussian blur (variance 0.25) + 30% missing pixels + 5% noise,
    CountSketch s = 101, rank 8, 30 steps: iterates within max(1e-8, 1e4 x the
    oracle's own spread) of the oracle's, the spread being the deviation of a
    second oracle run with the products summed in another order (~1e-12 after
    30 steps of the sketched solvers, ~4e-11 for FLSQR).  The factor 1e4: the
    GPU's truncated SVD stops at Ritz residuals of 1e-13 theta_1, some 1e3
    above the rounding of a full SVD, and the method amplifies either
    perturbation alike.  And z_K is the operator applied to the GPU's own p_K."""
    from paper_2605_22281_amd import sfk
    P = inputs.workload("deblur64")
    N, r, K = P.N, 8, 30
    say(f"case: deblur64 {method} {tau} r={r} K={K}")
    ctx, X, rho, rn, st = gpu_run(P, method, "sparse_sign", 101, K, zeta=1, seed=3001, tau=tau,
                                  lr_rows=N, lr_rank=r, stepwise=False)
    try:
        orc = _oracle(P, method, _oracle_tau(tau, N, r), K)
        orc2 = _oracle(P, method, _oracle_tau(tau, N, r), K, permuted=True)
        spread = np.maximum.accumulate([rel(orc2.X[:, j], orc.X[:, j]) for j in range(K)])
        assert X.shape[1] == K
        worst = 0.0
        for j in range(K):
            e = rel(X[:, j], orc.X[:, j])
            worst = max(worst, e)
            assert e <= max(1e-8, 1e4 * spread[j]), (j + 1, e, spread[j])
            if method != "flsqr":
                assert abs(rho[j] - orc.rho[j]) <= max(1e-8, 1e4 * spread[j]) * orc.rho[j]
        say(f"deblur64 {method} {tau}: worst rel err x over {K} steps {worst:.2e}, oracle "
            f"spread {spread[-1]:.1e}")
        # the last basis vector: z_K = tau(p_K) for the GPU's own p_K, rank <= r
        pk = sfk.basis_vector(ctx, "p", K).cpu().numpy()
        zk = sfk.basis_vector(ctx, "z", K).cpu().numpy()
        ref = (lowrank.truncate(pk, N, N, r) if tau == "lowrank"
               else lowrank.randomized_truncate(pk, N, N, r, seed=3001, call=K))
        assert rel(zk, ref) <= max(1e-10, _bound(pk.reshape(N, N), r)), rel(zk, ref)
        if tau == "lowrank":
            stt = sfk.tau_stats(ctx)
            say(f"  last call {stt['iterations']} power iterations, unconverged calls "
                f"{stt['unconverged_calls']}")
            assert stt["unconverged_calls"] == 0
    finally:
        sfk.destroy(ctx)


def test_lowrank_stop_and_stepwise_equal_batched():
    """Discrepancy stop with the low-rank operator; one call of 30 iterations
    and 30 calls of one give identical iterates (the operator is deterministic)."""
    from paper_2605_22281_amd import sfk
    P = inputs.workload("deblur64")
    N = P.N
    say("case: deblur64 lowrank discrepancy stop")
    c1, X1, _, _, _ = gpu_run(P, "sflsqr", "sparse_sign", 101, 30, zeta=1, tau="lowrank",
                              lr_rows=N, lr_rank=8, stepwise=True)
    c2, X2, _, _, _ = gpu_run(P, "sflsqr", "sparse_sign", 101, 30, zeta=1, tau="lowrank",
                              lr_rows=N, lr_rank=8, stepwise=False, **pinned(c1))
    sfk.destroy(c1)
    sfk.destroy(c2)
    assert np.array_equal(X1, X2)
    c3, X3, _, _, st = gpu_run(P, "sflsqr", "sparse_sign", 101, 60, zeta=1, tau="lowrank",
                               lr_rows=N, lr_rank=8, noise=P.noise_norm, eta=1.01)
    try:
        S = sketches.make("sparse_sign", P.m, 101, 3001, zeta=1)
        orc = fgk.sketched_flexible(P.A, P.b, S, maxit=60, tau=lowrank.Truncation(N, N, 8),
                                    tol=fgk.discrepancy_tol(1.01, P.noise_norm, np.linalg.norm(P.b)))
        assert c3.stopped == orc.stopped and X3.shape[1] == orc.k
    finally:
        sfk.destroy(c3)
