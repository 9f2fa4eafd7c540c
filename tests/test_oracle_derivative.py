"""The derivative oracle (oracle/derivative.py) against what fixes it
independently: its forward values are fgk.sketched_flexible's, and its
tangents equal central finite differences of the forward oracle (step h = 1e-6
relative), for b and eps, sFLSQR and sFLSMR, with the reweighting."""
import numpy as np
import pytest

from oracle import derivative, fgk, sketches
from paper_2605_22281_amd import inputs


def _problem(unmatched):
    return inputs.small_ct(16, 12, unmatched=unmatched, noise=0.02, phantom="sparse",
                           seed_offset=71)


@pytest.mark.parametrize("method,kind", [("sflsqr", "sparse_sign"), ("sflsmr", "srht")])
def test_forward_values_match_the_oracle(method, kind):
    P = _problem(method == "sflsmr")
    d = P.m if method == "sflsqr" else P.n
    S = sketches.make(kind, d, 50, 5)
    kw = dict(method=method, B=P.B, maxit=12, ell=2, tau="reweight_l1", eps=1e-2)
    X, dX = derivative.sketched_flexible_tangent(P.A, P.b, S, np.zeros(P.m), 0.0, **kw)
    orc = fgk.sketched_flexible(P.A, P.b, S, **kw)
    assert np.max(np.abs(X - orc.X)) <= 1e-14 * np.max(np.abs(orc.X))
    assert np.all(dX == 0.0)


@pytest.mark.parametrize("method,kind", [("sflsqr", "sparse_sign"), ("sflsmr", "srht")])
def test_tangent_equals_central_differences(method, kind):
    P = _problem(method == "sflsmr")
    d = P.m if method == "sflsqr" else P.n
    S = sketches.make(kind, d, 50, 5)
    eps = 1e-2
    kw = dict(method=method, B=P.B, maxit=12, ell=2, tau="reweight_l1")
    rng = np.random.default_rng(3)
    h = 1e-6
    nb = np.linalg.norm(P.b)
    for trial in range(6):
        db = rng.standard_normal(P.m)
        db *= nb / np.linalg.norm(db)
        deps = eps * rng.standard_normal() if trial % 2 else 0.0
        if trial == 5:
            db[:] = 0.0
            deps = eps
        L, dL = derivative.loss_tangent(P.A, P.b, S, P.x_true, db, deps, eps=eps, **kw)

        def loss(t):
            o = fgk.sketched_flexible(P.A, P.b + t * db, S, eps=eps + t * deps, **kw)
            e = o.X[:, -1] - P.x_true
            return 0.5 * float(e @ e)

        fd = (loss(h) - loss(-h)) / (2 * h)
        assert abs(fd - dL) <= 1e-6 * max(abs(dL), 1e-3 * L), (trial, fd, dL)


def test_tangent_is_linear_in_the_direction():
    P = _problem(False)
    S = sketches.make("sparse_sign", P.m, 50, 5)
    kw = dict(method="sflsqr", maxit=10, ell=2, tau="reweight_l1", eps=1e-2)
    rng = np.random.default_rng(4)
    d1, d2 = rng.standard_normal(P.m), rng.standard_normal(P.m)
    _, a = derivative.sketched_flexible_tangent(P.A, P.b, S, d1, 0.3, **kw)
    _, b = derivative.sketched_flexible_tangent(P.A, P.b, S, d2, -0.2, **kw)
    _, c = derivative.sketched_flexible_tangent(P.A, P.b, S, 2 * d1 + 3 * d2, 0.0, **kw)
    _, ce = derivative.sketched_flexible_tangent(P.A, P.b, S, np.zeros(P.m), 1.0, **kw)
    assert np.allclose(2 * a + 3 * b, c + (2 * 0.3 - 3 * 0.2) * ce, rtol=1e-9, atol=1e-12)
