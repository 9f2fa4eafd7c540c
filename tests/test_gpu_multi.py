"""Right-hand sides sharing one operator pair A, B: the long vectors of all of
them are interleaved and every product is one sparse-matrix-times-block pass.
Each right-hand side r (own b_r, own sketch seed, own stop test) must match the
CPU oracle run on it alone to the plain path's bar, and its own plain
single-instance GPU run."""
import numpy as np
import pytest
import torch

from oracle import fgk, sketches
from paper_2605_22281_amd import inputs

from gpu_cases import gpu_run, rel, rounding_spread, say

pytestmark = pytest.mark.gpu

MAXIT = 12

# (label, side, method, sketch, s, tau, R, unmatched B, stop test, vw); vw 2 stages
# the products through LDS (interleave widths 8, 16, 64 and 32 below), 0 gathers
CASES = [
    ("sflsqr-sparse_sign-R5-discrepancy", 24, "sflsqr", "sparse_sign", 90, "identity", 5, False, True, 2),
    ("sflsmr-srht-R9-unmatched-tol", 20, "sflsmr", "srht", 80, "identity", 9, True, True, 2),
    ("sflsqr-reweight-R4", 24, "sflsqr", "sparse_sign", 90, "reweight_l1", 4, False, False, 0),
    ("sflsqr-countsketch-R33-discrepancy", 16, "sflsqr", "countsketch", 60, "identity", 33, False, True, 2),
    ("sflsmr-reweight-R32-unmatched", 20, "sflsmr", "sparse_sign", 80, "reweight_l1", 32, True, False, 2),
    ("sflsqr-srht-R1", 16, "sflsqr", "srht", 50, "identity", 1, False, False, 0),
]


def _problem(side, unmatched, idx):
    na, nd = inputs.geometry_for_side(side)
    return inputs.ct_problem(side, max(na, 8), nd, noise=0.01, seed_offset=70 + idx,
                             unmatched=unmatched)


def _rhs_params(method, kind, s, tau, R, stop, dn, bnorm, vw=-2):
    """Per right-hand side: seed, discrepancy noise (sFLSQR) or tolerance (sFLSMR),
    chosen so that the right-hand sides stop at different iterations."""
    from paper_2605_22281_amd import sfk
    ps, tols = [], []
    for r in range(R):
        noise = tol = 0.0
        if stop and method == "sflsqr":
            noise = float(dn[r])
            tols.append(fgk.discrepancy_tol(1.01, noise, bnorm[r]))
        elif stop:
            tol = [1e-1, 3e-2, 1e-2, 0.0][r % 4]
            tols.append(tol)
        else:
            tols.append(0.0)
        ps.append(sfk.params(method, maxit=MAXIT, sketch=kind, s=s, seed=9000 + 7 * r, tau=tau,
                             eps=1e-2, noise_norm=noise, eta=1.01, tol=tol, vw=vw))
    return ps, tols


def _oracle(P, b, method, kind, s, tau, seed, tol):
    zeta = 1 if kind == "countsketch" else 8
    d = P.m if method == "sflsqr" else P.n
    S = sketches.make("sparse_sign" if kind == "countsketch" else kind, d, s, seed, zeta=zeta)
    return fgk.sketched_flexible(P.A, b, S, method=method, B=P.B, maxit=MAXIT, ell=2, tau=tau,
                                 eps=1e-2, tol=tol)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_shared_operator_rhs_match_oracle_and_plain(case):
    from paper_2605_22281_amd import sfk
    label, side, method, kind, s, tau, R, unmatched, stop, vw = case
    say("case:", label)
    P = _problem(side, unmatched, CASES.index(case))
    levels = [0.02 + 0.02 * (r % 5) for r in range(R)]   # 2% .. 10%
    b, xt, dn = inputs.multi_rhs(P, R, seed=11, noise=levels)
    bnorm = np.linalg.norm(b, axis=1)
    ps, tols = _rhs_params(method, kind, s, tau, R, stop, dn, bnorm, vw)
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B) if P.B is not None else None
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    ctx = sfk.init_multi(A, B, bb, ps)
    assert sfk.lib().sfk_batch_size(ctx.handle) == R
    assert sfk.spmv_variant(ctx) == ((-4, -4) if vw == 2 else (-2, -2))
    done, all_stopped, st = sfk.iterate(ctx, MAXIT)
    assert done == MAXIT
    ks = []
    # every right-hand side against the oracle; a sample against its plain GPU run
    sample = sorted({0, R // 2, R - 1})
    for r in range(R):
        k_r, stopped_r, brk = sfk.instance_status(ctx, r)
        orc = _oracle(P, b[r], method, kind, s, tau, 9000 + 7 * r, tols[r])
        assert (k_r, stopped_r) == (orc.k, orc.stopped), (r, k_r, stopped_r, orc.k, orc.stopped)
        x = sfk.instance_solution(ctx, r, P.n).cpu().numpy()
        rho, rn = sfk.instance_residual_norms(ctx, r, MAXIT)
        assert rel(x, orc.x) <= 1e-8, (r, rel(x, orc.x))
        assert abs(rn - orc.rhs_norm) <= 1e-12 * orc.rhs_norm
        for k in range(k_r):
            assert abs(rho[k] - orc.rho[k]) <= 1e-8 * orc.rho[k], (r, k)
        tr = sfk.instance_true_residual(ctx, r)
        assert abs(tr - np.linalg.norm(b[r] - P.A @ x)) <= 1e-10 * np.linalg.norm(b[r])
        ks.append(k_r)
        if r in sample:
            Pr = inputs.Problem(A=P.A, B=P.B, b=b[r], x_true=xt[r], noise_norm=float(dn[r]), N=P.N,
                                n_angles=P.n_angles, n_det=P.n_det)
            _, Xp, rhop, _, _ = gpu_run(Pr, method, kind, s, MAXIT, tau=tau, eps=1e-2,
                                        seed=9000 + 7 * r, zeta=1 if kind == "countsketch" else 8,
                                        noise=ps[r].noise_norm, tol=ps[r].tol, stepwise=False)
            assert Xp.shape[1] == k_r
            assert rel(x, Xp[:, -1]) <= 1e-9, (r, rel(x, Xp[:, -1]))
    say(f"{label}: iterations per right-hand side {ks}")
    if stop:
        assert len(set(ks)) > 1, "the stop tests should end the right-hand sides at different steps"


def test_shared_operator_resume_matches_one_call():
    from paper_2605_22281_amd import sfk
    say("case: shared-operator resume")
    P = _problem(20, False, 90)
    R = 6
    b, _, _ = inputs.multi_rhs(P, R, seed=12)
    A = sfk.to_device_csr(P.A)
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    ps = [sfk.params("sflsqr", maxit=10, s=70, seed=40 + r) for r in range(R)]
    c1 = sfk.init_multi(A, None, bb, ps)
    sfk.iterate(c1, 3)
    sfk.iterate(c1, 7)
    c2 = sfk.init_multi(A, None, bb, ps)
    sfk.iterate(c2, 10)
    for r in range(R):
        x1 = sfk.instance_solution(c1, r, P.n).cpu().numpy()
        x2 = sfk.instance_solution(c2, r, P.n).cpu().numpy()
        assert np.array_equal(x1, x2), r
        S = sketches.SparseSign(P.m, 70, 8, 40 + r)
        orc = fgk.sketched_flexible(P.A, b[r], S, maxit=10, ell=2)
        assert rel(x1, orc.x) <= 1e-8
    with pytest.raises(sfk.SfkError):
        sfk.iterate(c1, 1)


def test_shared_operator_invalid_arguments():
    from paper_2605_22281_amd import sfk
    say("case: shared-operator invalid arguments")
    P = _problem(16, False, 91)
    A = sfk.to_device_csr(P.A)
    b, _, _ = inputs.multi_rhs(P, 3, seed=13)
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    good = [sfk.params("sflsqr", maxit=8, s=60, seed=r) for r in range(3)]
    bad = list(good)
    bad[2] = sfk.params("sflsmr", maxit=8, s=60, seed=2)
    with pytest.raises(sfk.SfkError, match="method"):
        sfk.init_multi(A, None, bb, bad)
    bad = list(good)
    bad[1] = sfk.params("sflsqr", maxit=9, s=60, seed=1)
    with pytest.raises(sfk.SfkError, match="maxit"):
        sfk.init_multi(A, None, bb, bad)
    with pytest.raises(ValueError):
        sfk.init_multi(A, None, bb[:2], good)
    big = torch.zeros((65, P.m), dtype=torch.float64, device="cuda")
    with pytest.raises(sfk.SfkError):
        sfk.init_multi(A, None, big, [good[0]] * 65)
    zero = bb.clone()
    zero[1].zero_()
    with pytest.raises(sfk.SfkError, match="zero"):
        sfk.init_multi(A, None, zero, good)


def test_shared_operator_ct256_32_rhs():
    """256^2 CT, unmatched B, sFLSMR with SRHT s = 400, 32 right-hand sides (the
    batched throughput workload): sampled right-hand sides against the oracle
    through its reproducible horizon, all of them against their plain runs."""
    from paper_2605_22281_amd import sfk
    P = inputs.workload("ct256_unmatched")
    R, K = 32, 14
    say(f"case: ct256 shared operator, {R} right-hand sides, m={P.m} n={P.n}")
    b, xt, dn = inputs.multi_rhs(P, R, seed=21)
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B)
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    ps = [sfk.params("sflsmr", maxit=K, sketch="srht", s=400, seed=3100 + r) for r in range(R)]
    ctx = sfk.init_multi(A, B, bb, ps)
    done, _, _ = sfk.iterate(ctx, K)
    assert done == K
    for r in (0, 31):
        Pr = inputs.Problem(A=P.A, B=P.B, b=b[r], x_true=xt[r], noise_norm=float(dn[r]), N=P.N,
                            n_angles=P.n_angles, n_det=P.n_det)
        orc, spread = rounding_spread(Pr, "sflsmr", "srht", 400, K, seed=3100 + r)
        rho, _ = sfk.instance_residual_norms(ctx, r, K)
        x = sfk.instance_solution(ctx, r, P.n).cpu().numpy()
        horizon = 0
        for k in range(K):
            tol = max(1e-8, 1e3 * spread[k])
            er = abs(rho[k] - orc.rho[k]) / orc.rho[k]
            assert er <= tol, (r, k, er, tol)
            if tol == 1e-8:
                horizon = k + 1
        assert rel(x, orc.x) <= max(1e-8, 1e3 * spread[K - 1]), (r, rel(x, orc.x))
        say(f"ct256 rhs {r}: rho parity 1e-8 through k = {horizon}")
        assert horizon >= 10
    # every right-hand side against the oracle at 1e-8 through k = 10 (inside
    # the reproducible horizon of each of them)
    worst_o = 0.0
    for r in range(R):
        Pr = inputs.Problem(A=P.A, B=P.B, b=b[r], x_true=xt[r], noise_norm=float(dn[r]), N=P.N,
                            n_angles=P.n_angles, n_det=P.n_det)
        orc = fgk.sketched_flexible(P.A, b[r], sketches.SRHT(P.n, 400, 3100 + r), method="sflsmr",
                                    B=P.B, maxit=10, ell=2)
        rho, _ = sfk.instance_residual_norms(ctx, r, K)
        x10 = sfk.instance_solution_at(ctx, r, 10, P.n).cpu().numpy()
        er = np.max(np.abs(rho[:10] - orc.rho) / orc.rho)
        ex = rel(x10, orc.x)
        worst_o = max(worst_o, er, ex)
        assert er <= 1e-8 and ex <= 1e-8, (r, er, ex)
    say(f"ct256 32 rhs vs oracle, k <= 10: worst rel {worst_o:.2e}")
    ctx10 = sfk.init_multi(A, B, bb, [sfk.params("sflsmr", maxit=10, sketch="srht", s=400,
                                                 seed=3100 + r) for r in range(R)])
    sfk.iterate(ctx10, 10)
    worst = 0.0
    for r in range(R):
        Pr = inputs.Problem(A=P.A, B=P.B, b=b[r], x_true=xt[r], noise_norm=float(dn[r]), N=P.N,
                            n_angles=P.n_angles, n_det=P.n_det)
        x = sfk.instance_solution(ctx10, r, P.n).cpu().numpy()
        _, Xp, _, _, _ = gpu_run(Pr, "sflsmr", "srht", 400, 10, seed=3100 + r, stepwise=False)
        e = rel(x, Xp[:, -1])
        worst = max(worst, e)
        assert e <= 1e-8, (r, e)
    say(f"ct256 32 rhs vs plain runs at k=10: worst rel {worst:.2e}")


def test_shared_operator_row_kernel_matches_sliced():
    """The row kernel on the caller's CSR arrays (vw = -1), the column-sliced
    products gathering from L2 (vw = 0) or staged through LDS (vw = 2) and the
    automatic choice give the same iterates (all checked against the oracle)."""
    from paper_2605_22281_amd import sfk
    say("case: shared operator, row kernel vs sliced products")
    P = _problem(24, True, 92)
    R = 12
    b, _, _ = inputs.multi_rhs(P, R, seed=14)
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B)
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xs = {}
    expect = {0: (-2, -2), 2: (-4, -4), -1: (-3, -3)}
    for vw in (-2, 0, 2, -1):
        ps = [sfk.params("sflsmr", maxit=MAXIT, sketch="sparse_sign", s=90, seed=300 + r, vw=vw)
              for r in range(R)]
        ctx = sfk.init_multi(A, B, bb, ps)
        sfk.iterate(ctx, MAXIT)
        kern = sfk.spmv_variant(ctx)
        say(f"vw {vw}: kernels {kern}")
        assert kern == expect[vw] if vw in expect else set(kern) <= {-2, -4}
        xs[vw] = [sfk.instance_solution(ctx, r, P.n).cpu().numpy() for r in range(R)]
    for r in range(R):
        S = sketches.SparseSign(P.n, 90, 8, 300 + r)
        orc = fgk.sketched_flexible(P.A, b[r], S, method="sflsmr", B=P.B, maxit=MAXIT, ell=2)
        for vw in xs:
            assert rel(xs[vw][r], orc.x) <= 1e-8, (vw, r)
            assert rel(xs[vw][r], xs[-1][r]) <= 1e-10, (vw, r)
    # same partial slots and summation order inside a segment: staged and gathered agree
    for r in range(R):
        assert rel(xs[2][r], xs[0][r]) <= 1e-13, r


def test_shared_operator_ct256_staged_products():
    """256^2 CT in 4 x 4 pixel-tile order, 32 right-hand sides: the automatic
    choice stages B's products through LDS; every right-hand side matches the
    run that gathers from L2, and right-hand side 0 the oracle through its
    reproducible horizon."""
    from paper_2605_22281_amd import sfk
    P = inputs.workload("ct256_unmatched")
    R, K = 32, 12
    say(f"case: ct256 shared operator, tile order, staged vs gathered products, {R} right-hand sides")
    b, xt, dn = inputs.multi_rhs(P, R, seed=21)
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B)
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    perm = torch.from_numpy(inputs.tile_order(P.N, 4)).cuda()
    xs, rhos = {}, {}
    for vw in (-2, 0):
        ps = [sfk.params("sflsmr", maxit=K, sketch="srht", s=400, seed=3100 + r, vw=vw, perm=perm)
              for r in range(R)]
        ctx = sfk.init_multi(A, B, bb, ps)
        kern = sfk.spmv_variant(ctx)
        say(f"vw {vw}: kernels {kern}")
        assert kern[1] == (-4 if vw == -2 else -2)
        done, _, _ = sfk.iterate(ctx, K)
        assert done == K
        xs[vw] = [sfk.instance_solution(ctx, r, P.n).cpu().numpy() for r in range(R)]
        rhos[vw] = sfk.instance_residual_norms(ctx, 0, K)[0]
        sfk.destroy(ctx)
    worst = max(rel(xs[-2][r], xs[0][r]) for r in range(R))
    say(f"staged vs gathered at k = {K}: worst rel {worst:.2e}")
    assert worst <= 1e-10
    Pr = inputs.Problem(A=P.A, B=P.B, b=b[0], x_true=xt[0], noise_norm=float(dn[0]), N=P.N,
                        n_angles=P.n_angles, n_det=P.n_det)
    orc, spread = rounding_spread(Pr, "sflsmr", "srht", 400, K, seed=3100)
    horizon = 0
    for k in range(K):
        tol = max(1e-8, 1e3 * spread[k])
        er = abs(rhos[-2][k] - orc.rho[k]) / orc.rho[k]
        assert er <= tol, (k, er, tol)
        if tol == 1e-8:
            horizon = k + 1
    say(f"ct256 staged rhs 0: rho parity 1e-8 through k = {horizon}")
    assert horizon >= 10
