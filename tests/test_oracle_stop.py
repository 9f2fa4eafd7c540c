"""The oracle's stop rules against what eq. (discrP) and Algorithm 1 fix:
with true_tol the run ends at the first k with ||b - A x_k|| <= true_tol,
recomputed here from the returned iterates with a dense copy of A."""
import numpy as np
import pytest

from oracle import fgk, sketches
from paper_2605_22281_amd import inputs


@pytest.mark.parametrize("method", ["sflsqr", "sflsmr"])
def test_true_residual_stop_is_first_crossing(method):
    P = inputs.small_ct(20, 16, unmatched=True, noise=0.03)
    Ad = P.A.toarray()
    d = P.m if method == "sflsqr" else P.n
    S = sketches.SparseSign(d, 70, 8, 17)
    free = fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=40, ell=2)
    r = np.array([np.linalg.norm(P.b - Ad @ free.X[:, j]) for j in range(free.k)])
    assert np.allclose(r, free.res_true, rtol=1e-12)
    thr = 1.01 * P.noise_norm
    crossing = np.nonzero(r <= thr)[0]
    assert crossing.size > 0, "the discrepancy level is reached within 40 steps"
    kstop = int(crossing[0]) + 1
    orc = fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=40, ell=2, true_tol=thr)
    assert orc.stopped and orc.k == kstop
    assert np.array_equal(orc.X, free.X[:, :kstop])
    # not a sketched-test stop: the sketched objective at kstop is not what decides
    assert np.linalg.norm(P.b - Ad @ orc.x) <= thr
    assert np.all(r[: kstop - 1] > thr)


def test_one_stop_rule_at_a_time():
    P = inputs.small_ct(12, 10)
    S = sketches.SparseSign(P.m, 40, 4, 1)
    with pytest.raises(ValueError):
        fgk.sketched_flexible(P.A, P.b, S, maxit=5, tol=0.1, true_tol=1.0)
