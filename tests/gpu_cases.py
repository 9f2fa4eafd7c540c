"""Shared helpers of the GPU parity tests (not collected by pytest).

The GPU path is driven through the C ABI (paper_2605_22281_amd.sfk); the oracle
is the CPU float64 step-by-step implementation under oracle/.
"""
from __future__ import annotations

import sys

import numpy as np

from oracle import fgk, sketches


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_run(P, method, kind, s, maxit, *, ell=2, tau="identity", eps=1e-3, zeta=8, seed=3001,
            tol=0.0, noise=0.0, eta=1.01, stepwise=True, driver="auto", vw=-2, perm=None,
            resid=0, copies=0, **extra):
    """Runs the GPU solver; returns (ctx, X (n x k), rho, rhs_norm, status).
    perm: optional order of the unknowns (numpy int32, n entries); extra: more
    sfk.params keywords (the low-rank operator's lr_*)."""
    import torch
    from paper_2605_22281_amd import sfk
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B) if P.B is not None else None
    b = torch.from_numpy(np.ascontiguousarray(P.b)).cuda()
    pt = torch.from_numpy(np.ascontiguousarray(perm, dtype=np.int32)).cuda() if perm is not None else None
    p = sfk.params(method, ell=ell, maxit=maxit, sketch=kind, s=s, zeta=zeta, seed=seed, tau=tau,
                   eps=eps, tol=tol, noise_norm=noise, eta=eta, driver=driver, vw=vw, perm=pt,
                   resid=resid, copies=copies, **extra)
    ctx = sfk.init(A, B, b, p)
    X = []
    st = sfk.OK
    if stepwise:
        for _ in range(maxit):
            done, stopped, st = sfk.iterate(ctx, 1)
            if done > len(X):
                X.append(sfk.solution(ctx).cpu().numpy())
            if stopped or st != sfk.OK:
                break
    else:
        done, stopped, st = sfk.iterate(ctx, maxit)
        for j in range(1, done + 1):
            X.append(sfk.solution_at(ctx, j).cpu().numpy())
    rho, rn = sfk.residual_norms(ctx)
    Xm = np.stack(X, axis=1) if X else np.zeros((P.n, 0))
    return ctx, Xm, rho, rn, st


def pinned(ctx):
    """vw / vw_b that repeat the SpMV kernels ctx launches: the automatic
    choice is timed at init, so two contexts may differ in kernel and rounding."""
    from paper_2605_22281_amd import sfk
    va, vb = sfk.spmv_variant(ctx)
    return dict(vw=va, vw_b=vb)


def oracle_sketch(method, kind, P, s, zeta=8, seed=3001):
    d = P.m if method == "sflsqr" else P.n
    if kind == "identity":
        return sketches.Identity(d)
    return sketches.make(kind, d, s, seed, zeta=zeta)


def oracle_run(P, method, kind, s, maxit, *, ell=2, tau="identity", eps=1e-3, zeta=8, seed=3001,
               tol=0.0):
    S = oracle_sketch(method, kind, P, s, zeta, seed)
    return fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=maxit, ell=ell, tau=tau,
                                 eps=eps, tol=tol)


def compare(X, rho, orc, kmax, tol_x=1e-8, tol_rho=1e-8, label=""):
    """Element-by-element comparison of iterates and sketched residual norms."""
    worst_x = worst_r = 0.0
    for k in range(kmax):
        ex = rel(X[:, k], orc.X[:, k])
        er = abs(rho[k] - orc.rho[k]) / orc.rho[k]
        worst_x, worst_r = max(worst_x, ex), max(worst_r, er)
        assert ex <= tol_x, f"{label} x_{k + 1}: rel err {ex:.3e}"
        assert er <= tol_rho, f"{label} rho_{k + 1}: rel err {er:.3e}"
    say(f"{label}: k<={kmax} worst rel err x {worst_x:.2e} rho {worst_r:.2e}")
    return worst_x, worst_r


def rounding_spread(P, method, kind, s, maxit, *, ell=2, tau="identity", eps=1e-3, zeta=8,
                    seed=3001):
    """Deviation between two correctly rounded oracle runs that differ only in the
    summation order of the matrix-vector products (column permutation); its running
    maximum is the reproducibility floor of the method on this problem."""
    S = oracle_sketch(method, kind, P, s, zeta, seed)
    Bm = P.backprojector()
    r1 = fgk.sketched_flexible(P.A, P.b, S, method=method, B=Bm, maxit=maxit, ell=ell, tau=tau,
                               eps=eps)
    rng = np.random.default_rng(0)
    pc, pr = rng.permutation(P.n), rng.permutation(P.m)
    Ap = P.A[:, pc].tocsr()
    Ap.sort_indices()
    Bp = Bm[:, pr].tocsr()
    Bp.sort_indices()
    r2 = fgk.sketched_flexible(lambda v: Ap @ v[pc], P.b, S, method=method,
                               B=lambda v: Bp @ v[pr], maxit=maxit, ell=ell, tau=tau, eps=eps,
                               m=P.m, n=P.n)
    k = min(r1.k, r2.k)
    dev = np.array([max(rel(r2.X[:, j], r1.X[:, j]), abs(r2.rho[j] - r1.rho[j]) / r1.rho[j])
                    for j in range(k)])
    return r1, np.maximum.accumulate(dev)
