"""Step-by-step sFLSQR / sFLSMR and full-orthogonalisation FLSQR / FLSMR.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

Paper references (Bucci, Gazzola, Robol, "Randomized flexible LSQR and LSMR
with applications to inverse problems"):
  * flexible Golub-Kahan (FGK), eq. (flsqr-relations) and eq. (modbasis):
    A^T W_k = P_k T_k, A Z_k = W_{k+1} H_{k+1,k}, Z_k = tau(P_k);
  * FLSQR, eq. (FLSQR): y = argmin || ||b|| e_1 - H_{k+1,k} y ||;
  * FLSMR (Sec. 2.2): y = argmin || T_{k+1} (||b|| e_1 - H_{k+1,k} y) ||;
  * partially orthogonalised FGK, eq. (FGK), with window ell (Sec. 2.3);
  * sFLSQR, eq. (sFLSQR) and Algorithm 1: y = argmin || S(A Z_k y - b) ||;
  * sFLSMR, eq. (sFLSMR) and Algorithm 2: y = argmin || S(A^T A Z_k y - A^T b) ||,
    assembled as [S A^T W_k, S A^T w_{k+1}] H_{k+1,k};
  * discrepancy principle, eq. (discrP): ||A x_k - b|| <= eta * delta_e.

Readings where the paper is silent or inconsistent (all listed in the design
notes):
  * the z-side projections use the unit pre-tau vectors p_j (eq. (FGK) builds
    P with A^T W = P T and then Z = tau(P)); the algorithms' listings write z_j,
    which coincides when tau is the identity.  orth_against="Z" gives the
    literal variant (projection onto normalised z_j) for comparison;
  * modified Gram-Schmidt, ascending j, as the algorithms' loops are written;
  * the flexible operator for the l1 reweighting prior uses the previous
    iterate: z_k = (x_{k-1}^2 + eps^2)^(1/4) * p_k, with x_0 = 0;
  * stop test: sFLSQR uses Algorithm 1's test rho_k < tol * ||S b||; sFLSMR uses
    the minimised objective ||s - [S A^T W, S z] H y_k|| < tol * ||s|| (the
    listing's test drops the last column and H); with a discrepancy target the
    tolerance is tol = eta * delta_e / ||b||;
  * alternatively (true_tol > 0) the discrepancy principle on the true residual
    as eq. (discrP) writes it: stop at the first k with ||b - A x_k|| <= true_tol
    (= eta * delta_e), the sketched test then being off;
  * breakdown when t_kk <= 1e-14 * ||z before projection|| (basis cannot grow:
    return x_{k-1}) or h_{k+1,k} <= 1e-14 * ||A z_k|| (x_k is still formed with
    the new column, then the run stops);
  * the small least-squares problems are solved with a Householder QR
    (numpy.linalg.qr) and a triangular solve, recomputed from scratch each step.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

BREAKDOWN_TOL = 1e-14


def _matvec(M):
    if callable(M):
        return M
    return lambda v: M @ v


@dataclasses.dataclass
class Result:
    x: np.ndarray                     # final iterate
    k: int                            # iterations completed (index of x)
    stopped: bool                     # the stop test fired
    breakdown: bool
    X: np.ndarray                     # (n, k) iterates x_1..x_k
    rho: np.ndarray                   # (k,) minimised sketched objective
    rhs_norm: float                   # ||S b|| (sFLSQR) or ||S A^T b|| (sFLSMR)
    res_true: np.ndarray              # (k,) ||b - A x_j||
    H: np.ndarray                     # (k+1, k)
    T: np.ndarray                     # (k, k) (plus one column for FLSMR)
    P: np.ndarray                     # (n, k)
    Z: np.ndarray                     # (n, k)
    W: np.ndarray                     # (m, k+1)
    Ys: list                          # y_1..y_k
    beta: float


def lstsq_qr(M: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """argmin ||rhs - M y|| for full-column-rank M: Householder QR, back-substitution."""
    Q, R = np.linalg.qr(M, mode="reduced")
    return sla.solve_triangular(R, Q.T @ rhs, lower=False)


def tau_apply(tau, p: np.ndarray, x_prev: np.ndarray, eps: float, k: int = 0) -> np.ndarray:
    """Flexible operator for z_k = tau(p_k): identity, diagonal l1 reweighting
    (x_{k-1}^2 + eps^2)^(1/4), or a callable tau(p, x_prev, k) (the low-rank
    truncations of oracle.lowrank)."""
    if callable(tau):
        return np.asarray(tau(p, x_prev, k), dtype=np.float64)
    if tau == "identity":
        return p.copy()
    if tau == "reweight_l1":
        return np.sqrt(np.sqrt(x_prev * x_prev + eps * eps)) * p
    raise ValueError(tau)


def sketched_flexible(A, b, sketch, *, method: str = "sflsqr", B=None, maxit: int = 50,
                      ell: int = 2, tau: str = "identity", eps: float = 1e-3,
                      tol: float = 0.0, orth_against: str = "P", m: int | None = None,
                      n: int | None = None, true_tol: float = 0.0) -> Result:
    """sFLSQR (Algorithm 1) or sFLSMR (Algorithm 2), step by step.

    A, B: matrices (dense or scipy sparse) or callables; B None means A^T.
    sketch: object with .apply(v) -> S v (S acts on m-vectors for sFLSQR and on
    n-vectors for sFLSMR).
    true_tol: > 0 stops on ||b - A x_k|| <= true_tol instead of the sketched test.
    """
    if true_tol > 0.0 and tol > 0.0:
        raise ValueError("one stop test at a time: tol (sketched) or true_tol")
    if method not in ("sflsqr", "sflsmr"):
        raise ValueError(method)
    Av = _matvec(A)
    if B is None:
        if callable(A):
            raise ValueError("B required when A is a callable")
        AT = A.T
        Bv = lambda v: AT @ v
    else:
        Bv = _matvec(B)
    b = np.asarray(b, dtype=np.float64)
    m = b.shape[0] if m is None else m

    # initialisation (Alg. 1 / Alg. 2, first lines)
    beta = float(np.linalg.norm(b))
    w1 = b / beta
    z = Bv(w1)
    n = z.shape[0] if n is None else n
    if method == "sflsqr":
        s_rhs = sketch.apply(b)
        SAZ = []
    else:
        c = sketch.apply(z)
        s_rhs = beta * c
        SBW = [c]
    rhs_norm = float(np.linalg.norm(s_rhs))

    W = [w1]
    P, Z = [], []
    H = np.zeros((maxit + 1, maxit))
    T = np.zeros((maxit, maxit))
    x_prev = np.zeros(n)
    X, rhos, rtrue, Ys = [], [], [], []
    stopped = breakdown = False
    k_done = 0

    for k in range(1, maxit + 1):
        # truncated MGS of z against the last ell basis vectors (window j = k-ell .. k-1)
        z_pre_norm = float(np.linalg.norm(z))
        for j in range(max(1, k - ell), k):
            if orth_against == "P":
                q = P[j - 1]
                t = float(np.dot(q, z))
                z = z - t * q
            else:
                q = Z[j - 1] / np.linalg.norm(Z[j - 1])
                t = float(np.dot(q, z))
                z = z - t * q
            T[j - 1, k - 1] = t
        tkk = float(np.linalg.norm(z))
        if tkk <= BREAKDOWN_TOL * z_pre_norm or tkk == 0.0:
            breakdown = True
            break
        T[k - 1, k - 1] = tkk
        p = z / tkk
        P.append(p)
        zk = tau_apply(tau, p, x_prev, eps, k)
        Z.append(zk)

        w = Av(zk)
        if method == "sflsqr":
            SAZ.append(sketch.apply(w))
        w_pre_norm = float(np.linalg.norm(w))
        # truncated MGS of w against w_j, j = k-ell .. k
        for j in range(max(1, k - ell), k + 1):
            h = float(np.dot(W[j - 1], w))
            w = w - h * W[j - 1]
            H[j - 1, k - 1] = h
        hk = float(np.linalg.norm(w))
        happy = hk <= BREAKDOWN_TOL * w_pre_norm or hk == 0.0
        if happy:
            hk = 0.0
            w = np.zeros_like(w)
            H[k, k - 1] = 0.0
            W.append(w)
            z = np.zeros(n)
        else:
            H[k, k - 1] = hk
            w = w / hk
            W.append(w)
            z = Bv(w)

        # small sketched least-squares problem
        if method == "sflsqr":
            M = np.stack(SAZ, axis=1)
        else:
            c = sketch.apply(z) if not happy else np.zeros_like(s_rhs)
            M = np.stack(SBW + [c], axis=1) @ H[: k + 1, :k]
        y = lstsq_qr(M, s_rhs)
        rho = float(np.linalg.norm(s_rhs - M @ y))
        Zm = np.stack(Z, axis=1)
        x = Zm @ y
        X.append(x)
        Ys.append(y)
        rhos.append(rho)
        rtrue.append(float(np.linalg.norm(b - Av(x))))
        k_done = k
        x_prev = x
        if method == "sflsmr":
            SBW.append(c)
        if happy:
            breakdown = True
            break
        if tol > 0.0 and rho < tol * rhs_norm:
            stopped = True
            break
        if true_tol > 0.0 and rtrue[-1] <= true_tol:
            stopped = True
            break

    k = k_done
    Xm = np.stack(X, axis=1) if X else np.zeros((n, 0))
    return Result(
        x=X[-1] if X else np.zeros(n), k=k, stopped=stopped, breakdown=breakdown, X=Xm,
        rho=np.array(rhos), rhs_norm=rhs_norm, res_true=np.array(rtrue),
        H=H[: k + 1, :k], T=T[:k, :k],
        P=np.stack(P[:k], axis=1) if k else np.zeros((n, 0)),
        Z=np.stack(Z[:k], axis=1) if k else np.zeros((n, 0)),
        W=np.stack(W[: k + 1], axis=1), Ys=Ys, beta=beta)


def discrepancy_tol(eta: float, noise_norm: float, beta: float) -> float:
    """Relative tolerance of the sketched test that stands for ||A x - b|| <= eta delta_e."""
    return eta * noise_norm / beta


def flexible_full(A, b, *, method: str = "flsqr", B=None, maxit: int = 20,
                  tau: str = "identity", eps: float = 1e-3) -> Result:
    """FLSQR / FLSMR with full orthogonalisation (Sec. 2.2), without sketching.

    FLSQR:  y = argmin || beta e_1 - H_{k+1,k} y ||            (eq. (FLSQR))
    FLSMR:  y = argmin || T_{k+1} (beta e_1 - H_{k+1,k} y) ||
    Both rely on the orthonormality of W and P produced by full MGS.
    """
    Av = _matvec(A)
    if B is None:
        AT = A.T
        Bv = lambda v: AT @ v
    else:
        Bv = _matvec(B)
    b = np.asarray(b, dtype=np.float64)
    beta = float(np.linalg.norm(b))
    W = [b / beta]
    z = Bv(W[0])
    n = z.shape[0]
    P, Z = [], []
    H = np.zeros((maxit + 1, maxit))
    T = np.zeros((maxit + 1, maxit + 1))
    x_prev = np.zeros(n)
    X, rhos, rtrue, Ys = [], [], [], []

    def orth_z(z, k):
        # full MGS of z against p_1..p_{k-1}; fills column k of T (1-based)
        for j in range(1, k):
            t = float(np.dot(P[j - 1], z))
            z = z - t * P[j - 1]
            T[j - 1, k - 1] = t
        tkk = float(np.linalg.norm(z))
        T[k - 1, k - 1] = tkk
        return z / tkk

    p = orth_z(z, 1)
    for k in range(1, maxit + 1):
        P.append(p)
        zk = tau_apply(tau, p, x_prev, eps, k)
        Z.append(zk)
        w = Av(zk)
        for j in range(1, k + 1):
            h = float(np.dot(W[j - 1], w))
            w = w - h * W[j - 1]
            H[j - 1, k - 1] = h
        hk = float(np.linalg.norm(w))
        H[k, k - 1] = hk
        W.append(w / hk)
        z = Bv(W[-1])
        p_next = orth_z(z, k + 1)          # gives column k+1 of T
        e1 = np.zeros(k + 1)
        e1[0] = beta
        Hk = H[: k + 1, :k]
        if method == "flsqr":
            y = lstsq_qr(Hk, e1)
            rho = float(np.linalg.norm(e1 - Hk @ y))
        else:
            Tk1 = T[: k + 1, : k + 1]
            y = lstsq_qr(Tk1 @ Hk, Tk1 @ e1)
            rho = float(np.linalg.norm(Tk1 @ (e1 - Hk @ y)))
        x = np.stack(Z, axis=1) @ y
        X.append(x)
        Ys.append(y)
        rhos.append(rho)
        rtrue.append(float(np.linalg.norm(b - Av(x))))
        x_prev = x
        p = p_next
    return Result(x=X[-1], k=maxit, stopped=False, breakdown=False, X=np.stack(X, axis=1),
                  rho=np.array(rhos), rhs_norm=beta, res_true=np.array(rtrue),
                  H=H[: maxit + 1, :maxit], T=T[: maxit + 1, : maxit + 1],
                  P=np.stack(P, axis=1), Z=np.stack(Z, axis=1), W=np.stack(W, axis=1),
                  Ys=Ys, beta=beta)
