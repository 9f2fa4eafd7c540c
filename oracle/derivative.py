"""Derivative of the sFLSQR / sFLSMR iterate x_k with respect to the
right-hand side b and the reweighting parameter eps (forward mode).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

x_k is defined by the recurrences of eq. (FGK) (partial Gram-Schmidt with
window ell, normalisation, the flexible operator tau of eq. (modbasis), here
the l1 reweighting z_k = (x_{k-1}^2 + eps^2)^(1/4) p_k) and the small sketched
least-squares problem of eq. (sFLSQR) / eq. (sFLSMR).  Every step is a smooth
function of b and eps (away from breakdowns), so the chain rule carries a
tangent (db, deps) through each of them in the same order: for a scalar
product t = <p, z> the tangent is <dp, z> + <p, dz>, for a norm r = ||u|| it
is <u, du> / r, for the reweighting
  d (x^2 + eps^2)^(1/4) = (x dx + eps deps) / (2 (x^2 + eps^2)^(3/4)),
and for the least-squares solution y = argmin ||s - M y|| of a full column
rank M with residual r = s - M y
  dy = (M^T M)^{-1} (M^T (ds - dM y) + dM^T r).
The forward values are computed alongside, with the same operations in the
same order as fgk.sketched_flexible (test_oracle_derivative checks that they
agree), and the tangent of 0.5 ||x_k - x_true||^2 along (db, deps) is
<x_k - x_true, dx_k>.  The test pins it to central finite differences of the
forward oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _mv(M):
    return M if callable(M) else (lambda v: M @ v)


def _lstsq_with_tangent(M, dM, s, ds):
    Q, R = np.linalg.qr(M, mode="reduced")
    y = sla.solve_triangular(R, Q.T @ s, lower=False)
    r = s - M @ y
    g = Q.T @ (ds - dM @ y)
    dy = sla.solve_triangular(R, g, lower=False)
    # (M^T M)^{-1} dM^T r = R^{-1} R^{-T} dM^T r
    u = sla.solve_triangular(R, dM.T @ r, trans="T", lower=False)
    dy = dy + sla.solve_triangular(R, u, lower=False)
    return y, dy, r


def sketched_flexible_tangent(A, b, sketch, db, deps, *, method="sflsqr", B=None,
                              maxit=50, ell=2, tau="reweight_l1", eps=1e-3):
    """Iterates x_1..x_maxit and their tangents along (db, deps).

    Returns (X, dX) with columns x_k, dx_k.  No stop test: the derivative of a
    fixed number of steps (breakdowns raise)."""
    Av = _mv(A)
    if B is None:
        AT = A.T
        Bv = lambda v: AT @ v
    else:
        Bv = _mv(B)
    Sv = sketch.apply
    b = np.asarray(b, dtype=np.float64)
    db = np.asarray(db, dtype=np.float64)

    beta = float(np.linalg.norm(b))
    dbeta = float(b @ db) / beta
    w = b / beta
    dw = (db - w * dbeta) / beta
    z, dz = Bv(w), Bv(dw)
    n = z.shape[0]
    if method == "sflsqr":
        s_rhs, ds_rhs = Sv(b), Sv(db)
        C, dC = [], []
    else:
        c, dc = Sv(z), Sv(dz)
        s_rhs, ds_rhs = beta * c, dbeta * c + beta * dc
        SBW, dSBW = [c], [dc]
    W, dW = [w], [dw]
    P, dP, Z, dZ = [], [], [], []
    H = np.zeros((maxit + 1, maxit))
    dH = np.zeros((maxit + 1, maxit))
    x_prev, dx_prev = np.zeros(n), np.zeros(n)
    X, dX = [], []
    for k in range(1, maxit + 1):
        # z-side: window j = max(1, k - ell) .. k - 1 against the unit p_j
        for j in range(max(1, k - ell), k):
            p, dp = P[j - 1], dP[j - 1]
            t = float(p @ z)
            dt = float(dp @ z) + float(p @ dz)
            z, dz = z - t * p, dz - dt * p - t * dp
        tkk = float(np.linalg.norm(z))
        if tkk == 0.0:
            raise ZeroDivisionError("breakdown")
        dtkk = float(z @ dz) / tkk
        p = z / tkk
        dp = (dz - p * dtkk) / tkk
        P.append(p)
        dP.append(dp)
        if tau == "identity":
            zk, dzk = p.copy(), dp.copy()
        elif tau == "reweight_l1":
            q = x_prev * x_prev + eps * eps
            d = np.sqrt(np.sqrt(q))
            dd = (x_prev * dx_prev + eps * deps) * d / (2.0 * q)     # = (...) / (2 q^(3/4))
            zk, dzk = d * p, dd * p + d * dp
        else:
            raise ValueError(tau)
        Z.append(zk)
        dZ.append(dzk)
        v, dv = Av(zk), Av(dzk)
        if method == "sflsqr":
            C.append(Sv(v))
            dC.append(Sv(dv))
        # w-side: window j = max(1, k - ell) .. k against w_j
        for j in range(max(1, k - ell), k + 1):
            wj, dwj = W[j - 1], dW[j - 1]
            h = float(wj @ v)
            dh = float(dwj @ v) + float(wj @ dv)
            H[j - 1, k - 1], dH[j - 1, k - 1] = h, dh
            v, dv = v - h * wj, dv - dh * wj - h * dwj
        hk = float(np.linalg.norm(v))
        if hk == 0.0:
            raise ZeroDivisionError("happy breakdown")
        dhk = float(v @ dv) / hk
        H[k, k - 1], dH[k, k - 1] = hk, dhk
        w = v / hk
        dw = (dv - w * dhk) / hk
        W.append(w)
        dW.append(dw)
        z, dz = Bv(w), Bv(dw)
        if method == "sflsqr":
            M, dM = np.stack(C, axis=1), np.stack(dC, axis=1)
        else:
            c, dc = Sv(z), Sv(dz)
            Sm = np.stack(SBW + [c], axis=1)
            dSm = np.stack(dSBW + [dc], axis=1)
            M = Sm @ H[: k + 1, :k]
            dM = dSm @ H[: k + 1, :k] + Sm @ dH[: k + 1, :k]
        y, dy, _ = _lstsq_with_tangent(M, dM, s_rhs, ds_rhs)
        Zm, dZm = np.stack(Z, axis=1), np.stack(dZ, axis=1)
        x = Zm @ y
        dx = dZm @ y + Zm @ dy
        X.append(x)
        dX.append(dx)
        x_prev, dx_prev = x, dx
        if method == "sflsmr":
            SBW.append(c)
            dSBW.append(dc)
    return np.stack(X, axis=1), np.stack(dX, axis=1)


def loss_tangent(A, b, sketch, x_true, db, deps, **kw):
    """(L, dL) for L = 0.5 ||x_K - x_true||^2, K = kw['maxit'], along (db, deps)."""
    X, dX = sketched_flexible_tangent(A, b, sketch, db, deps, **kw)
    e = X[:, -1] - x_true
    return 0.5 * float(e @ e), float(e @ dX[:, -1])
