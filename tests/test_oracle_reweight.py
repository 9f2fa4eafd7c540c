"""Pins of the oracle's flexible operator for the l1 reweighting prior.

Sec. 1 of the paper presents sparsity priors through iteratively reweighted
least squares (IRLS): the inverses of the weights that approximate the
(semi)norm act as variable right preconditioners.  For the smoothed l1 norm
phi(x) = sum_i sqrt(x_i^2 + eps^2), the IRLS quadratic that touches phi at
xhat has the diagonal weight phi'(xhat_i) / xhat_i (phi''(0) at xhat_i = 0);
writing the penalty as ||W x||^2, the right preconditioner is W^{-1}, i.e.
d_i = (phi'(xhat_i) / xhat_i)^(-1/2).  The weights below are derived from phi
itself by central differences, not from the oracle's formula, and the
oracle's basis must satisfy z_k = d(x_{k-1}) * p_k with x_0 = 0:

  * k = 1: d = eps^(1/2) exactly (a closed form; an exponent of 1/2 on
    (x^2 + eps^2) would give eps, and a weight built from x_1 would not be
    constant);
  * k >= 2: the weight is the one of x_{k-1}, and it is not the one of x_k.
"""
import numpy as np
import pytest

from oracle import fgk, sketches
from paper_2605_22281_amd import inputs


def phi(x, eps):
    return np.sqrt(x * x + eps * eps)


def irls_inverse_weight(xhat, eps):
    """d_i = (phi'(xhat_i) / xhat_i)^(-1/2), phi' by central differences; at
    xhat_i = 0 the ratio's limit phi''(0) by a second difference."""
    xhat = np.asarray(xhat, dtype=np.float64)
    out = np.empty_like(xhat)
    big = np.abs(xhat) >= 1e-3 * eps
    h = 1e-6 * np.maximum(eps, np.abs(xhat[big]))
    dphi = (phi(xhat[big] + h, eps) - phi(xhat[big] - h, eps)) / (2.0 * h)
    out[big] = (dphi / xhat[big]) ** -0.5
    small = ~big
    if np.any(small):
        x0 = xhat[small]
        h2 = 1e-3 * eps
        d2 = (phi(x0 + h2, eps) - 2.0 * phi(x0, eps) + phi(x0 - h2, eps)) / (h2 * h2)
        out[small] = d2 ** -0.5
    return out


@pytest.fixture(scope="module")
def problem():
    return inputs.small_ct(16, 12, noise=0.02, phantom="sparse", seed_offset=31)


def _run(P, eps, maxit=6):
    S = sketches.SparseSign(P.m, 80, 8, 17)
    return fgk.sketched_flexible(P.A, P.b, S, maxit=maxit, ell=2, tau="reweight_l1", eps=eps)


@pytest.mark.parametrize("eps", [1e-3, 0.25, 4.0])
def test_first_weight_is_sqrt_eps(problem, eps):
    r = _run(problem, eps, maxit=1)
    z1, p1 = r.Z[:, 0], r.P[:, 0]
    assert np.linalg.norm(p1) == pytest.approx(1.0, rel=1e-14)
    # x_0 = 0: (0 + eps^2)^(1/4) = sqrt(eps), the same for every entry
    np.testing.assert_allclose(z1, np.sqrt(eps) * p1, rtol=1e-15, atol=0.0)
    # and the derivative-based IRLS weight of x_0 = 0 agrees
    d0 = irls_inverse_weight(np.zeros(problem.n), eps)
    np.testing.assert_allclose(d0, np.sqrt(eps), rtol=1e-5)


@pytest.mark.parametrize("eps", [0.02, 0.3])
def test_later_weights_come_from_previous_iterate(problem, eps):
    r = _run(problem, eps, maxit=6)
    assert r.k == 6
    for k in range(2, r.k + 1):
        p, z = r.P[:, k - 1], r.Z[:, k - 1]
        x_prev, x_cur = r.X[:, k - 2], r.X[:, k - 1]
        d_prev = irls_inverse_weight(x_prev, eps)
        d_cur = irls_inverse_weight(x_cur, eps)
        ok = np.abs(p) > 1e-12 * np.abs(p).max()
        ratio = z[ok] / p[ok]
        err_prev = np.max(np.abs(ratio - d_prev[ok]) / d_prev[ok])
        err_cur = np.max(np.abs(ratio - d_cur[ok]) / d_cur[ok])
        assert err_prev < 1e-6, (k, err_prev)
        # the weight of x_k itself is measurably different
        assert err_cur > 1e-3, (k, err_cur)


def test_weight_is_not_inverse_irls_weight(problem):
    """The preconditioner is W^{-1} (weights to the power -1/2 of phi'(x)/x), not
    W^{-2} = (x^2 + eps^2)^(1/2): on an iterate with entries far from zero the
    two differ by orders of magnitude."""
    eps = 1e-3
    r = _run(problem, eps, maxit=3)
    x1 = r.X[:, 0]
    z2, p2 = r.Z[:, 1], r.P[:, 1]
    ok = (np.abs(p2) > 1e-12 * np.abs(p2).max()) & (np.abs(x1) > 5 * eps)
    assert ok.sum() > 10
    wrong = np.sqrt(x1[ok] ** 2 + eps ** 2)
    assert np.max(np.abs(z2[ok] / p2[ok] - wrong) / wrong) > 0.1
