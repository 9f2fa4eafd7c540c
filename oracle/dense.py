"""Definitional dense forms and the paper's bounds, for tiny problems.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

  * eq. (sFLSQR): x_k = Z_k y, y = argmin || S A Z_k y - S b ||
  * eq. (sFLSMR): x_k = Z_k y, y = argmin || S A^T A Z_k y - S A^T b ||
    (with an unmatched back-projector B in place of A^T)
  * Theorem 1: r^sFLSQR <= r^opt sqrt(1 + ||(S Q)^+ S Q_perp||^2) and
    r^sFLSMR <= r^opt sqrt(1 + ||(S A^T Q)^+ S A^T Q_perp||^2), Q an orthonormal
    basis of range(A Z_k), Q_perp of its complement, r^opt the optimal residual
    norm over range(Z_k)
  * Corollary 1 (Gaussian S, entries N(0, 1)):
    E[(r^sFLSQR)^2] = (r^opt)^2 (1 + k / (s - k - 1)).  The printed numerator
    is s; Halko-Martinsson-Tropp Prop. 10.2 gives E||G^+||_F^2 = k / (s - k - 1)
    for a Gaussian s x k matrix G, which is the form used here.
"""
from __future__ import annotations

import numpy as np


def dense(M):
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M, dtype=np.float64)


def sflsqr_from_basis(A, b, S: np.ndarray, Z: np.ndarray) -> np.ndarray:
    A = dense(A)
    y = np.linalg.lstsq(S @ A @ Z, S @ b, rcond=None)[0]
    return Z @ y


def sflsmr_from_basis(A, b, S: np.ndarray, Z: np.ndarray, B=None) -> np.ndarray:
    A = dense(A)
    Bm = A.T if B is None else dense(B)
    y = np.linalg.lstsq(S @ Bm @ A @ Z, S @ Bm @ b, rcond=None)[0]
    return Z @ y


def optimal_residual(A, b, Z: np.ndarray) -> float:
    A = dense(A)
    y = np.linalg.lstsq(A @ Z, b, rcond=None)[0]
    return float(np.linalg.norm(A @ Z @ y - b))


def theorem1_bounds(A, b, Z: np.ndarray, S_m: np.ndarray | None = None,
                    S_n: np.ndarray | None = None, B=None):
    """(r_opt, bound of eq. (bound1), bound of eq. (bound2)) of Theorem 1.

    S_m sketches m-vectors (sFLSQR), S_n sketches n-vectors (sFLSMR); a bound whose
    sketch is not given is returned as nan.
    """
    A = dense(A)
    Bm = A.T if B is None else dense(B)
    k = Z.shape[1]
    Qfull, _ = np.linalg.qr(A @ Z, mode="complete")
    Q, Qp = Qfull[:, :k], Qfull[:, k:]
    r_opt = float(np.linalg.norm(Qp.T @ b))
    b1 = b2 = float("nan")
    if S_m is not None:
        g1 = np.linalg.norm(np.linalg.pinv(S_m @ Q) @ (S_m @ Qp), 2)
        b1 = r_opt * np.sqrt(1.0 + g1 ** 2)
    if S_n is not None:
        g2 = np.linalg.norm(np.linalg.pinv(S_n @ Bm @ Q) @ (S_n @ Bm @ Qp), 2)
        b2 = r_opt * np.sqrt(1.0 + g2 ** 2)
    return r_opt, b1, b2


def corollary1_factor(k: int, s: int) -> float:
    return 1.0 + k / (s - k - 1.0)
