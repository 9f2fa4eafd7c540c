"""Batched mode: independent instances of uneven sizes in one context, each
stage kernel serving all of them in one launch, per-instance stopping.  Every
instance must match the CPU oracle (and its own plain single-instance run) to
the same bar as the plain path."""
import numpy as np
import pytest
import torch

from oracle import fgk, sketches
from paper_2605_22281_amd import inputs

from gpu_cases import compare, gpu_run, rel, say

pytestmark = pytest.mark.gpu

# (side, method, sketch, s, tau, discrepancy)
CASES = [
    (16, "sflsqr", "sparse_sign", 60, "identity", True),
    (24, "sflsmr", "srht", 80, "identity", False),
    (32, "sflsqr", "sparse_sign", 90, "reweight_l1", False),
    (20, "sflsqr", "countsketch", 70, "identity", True),
    (28, "sflsmr", "sparse_sign", 100, "reweight_l1", False),
    (12, "sflsqr", "srht", 40, "identity", False),
]
MAXIT = 12


def _problems():
    out = []
    for i, (side, *_rest) in enumerate(CASES):
        na, nd = inputs.geometry_for_side(side)
        P = inputs.ct_problem(side, max(na, 8), nd, noise=0.01 + 0.004 * i, seed_offset=50 + i,
                              unmatched=(i % 2 == 1))
        out.append(P)
    return out


def _oracle(P, method, kind, s, tau, disc, seed):
    zeta = 1 if kind == "countsketch" else 8
    d = P.m if method == "sflsqr" else P.n
    S = sketches.make("sparse_sign" if kind == "countsketch" else kind, d, s, seed, zeta=zeta)
    tol = fgk.discrepancy_tol(1.01, P.noise_norm, np.linalg.norm(P.b)) if disc else 0.0
    return fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=MAXIT, ell=2, tau=tau,
                                 eps=1e-2, tol=tol)


def test_heterogeneous_batch_matches_oracle_and_plain():
    from paper_2605_22281_amd import sfk
    probs = _problems()
    say("case: heterogeneous batch of", len(probs))
    As, Bs, bs, ps = [], [], [], []
    for i, (P, (side, method, kind, s, tau, disc)) in enumerate(zip(probs, CASES)):
        As.append(sfk.to_device_csr(P.A))
        Bs.append(sfk.to_device_csr(P.B) if P.B is not None else None)
        bs.append(torch.from_numpy(P.b).cuda())
        ps.append(sfk.params(method, maxit=MAXIT, sketch=kind, s=s, seed=7000 + i, tau=tau, eps=1e-2,
                             noise_norm=P.noise_norm if disc else 0.0, eta=1.01))
    ctx = sfk.init_batch(As, Bs, bs, ps)
    done, all_stopped, st = sfk.iterate(ctx, MAXIT)
    assert done == MAXIT
    for i, (P, (side, method, kind, s, tau, disc)) in enumerate(zip(probs, CASES)):
        k_i, stopped_i, brk = sfk.instance_status(ctx, i)
        orc = _oracle(P, method, kind, s, tau, disc, 7000 + i)
        assert k_i == orc.k and stopped_i == orc.stopped, (i, k_i, orc.k)
        x = sfk.instance_solution(ctx, i, P.n).cpu().numpy()
        rho, rn = sfk.instance_residual_norms(ctx, i, MAXIT)
        assert rel(x, orc.x) <= 1e-8, (i, rel(x, orc.x))
        for k in range(k_i):
            assert abs(rho[k] - orc.rho[k]) <= 1e-8 * orc.rho[k], (i, k)
        # same instance on its own
        _, Xp, rhop, _, _ = gpu_run(P, method, kind, s, MAXIT, tau=tau, eps=1e-2, seed=7000 + i,
                                    zeta=1 if kind == "countsketch" else 8,
                                    noise=P.noise_norm if disc else 0.0, stepwise=False)
        assert Xp.shape[1] == k_i
        assert rel(x, Xp[:, -1]) <= 1e-10
        say(f"instance {i} side {side} {method}/{kind}/{tau}: k={k_i} stopped={stopped_i} "
            f"rel err {rel(x, orc.x):.1e}")


def test_batch_resume_and_per_instance_capacity():
    from paper_2605_22281_amd import sfk
    probs = _problems()[:3]
    say("case: batch resume with unequal maxit")
    As = [sfk.to_device_csr(P.A) for P in probs]
    bs = [torch.from_numpy(P.b).cuda() for P in probs]
    caps = [5, 9, 7]
    ps = [sfk.params("sflsqr", maxit=c, s=60, seed=11 + i) for i, c in enumerate(caps)]
    ctx = sfk.init_batch(As, None, bs, ps)
    sfk.iterate(ctx, 4)
    sfk.iterate(ctx, 5)
    for i, P in enumerate(probs):
        k_i, _, _ = sfk.instance_status(ctx, i)
        assert k_i == caps[i]
        S = sketches.SparseSign(P.m, 60, 8, 11 + i)
        orc = fgk.sketched_flexible(P.A, P.b, S, maxit=caps[i], ell=2)
        x = sfk.instance_solution(ctx, i, P.n).cpu().numpy()
        assert rel(x, orc.x) <= 1e-8
    with pytest.raises(sfk.SfkError):
        sfk.iterate(ctx, 1)            # largest capacity (9) exhausted


@pytest.mark.skip(reason="this case failed in a run that left the GPU with a memory fault "
                  "(together with a change to the least-squares kernels that read no address "
                  "the current kernels do not, since taken out); the cause has not been shown, "
                  "so the case stays off the GPU until it is")
def test_heterogeneous_batch_at_benchmark_sizes():
    """The heterogeneous benchmark's batch at its own sizes: its first four
    instances (one of each side 256, 128, 384, 192; 1.9e6 to 5.1e7 nonzeros),
    4 x 4 tile order, sFLSQR, sparse-sign s = 201, discrepancy stop eta = 1.01.
    Each instance's stopping iteration, x at the stop and rho_k against the
    oracle (1e-8; the stops come before the reproducibility horizon), and
    against the same instance solved on its own."""
    from paper_2605_22281_amd import sfk
    count, sel = 32, [0, 1, 2, 3]
    drawn = inputs.batch_instance_sides(count)
    assert sorted(drawn[i][0] for i in sel) == [128, 192, 256, 384]
    probs = inputs.batch_instances(count, select=sel)
    say("case: heterogeneous batch at the benchmark sizes, sides", [P.N for P in probs])
    perms = [inputs.tile_order(P.N, 4) for P in probs]
    As = [sfk.to_device_csr(P.A) for P in probs]
    bs = [torch.from_numpy(np.ascontiguousarray(P.b)).cuda() for P in probs]
    pts = [torch.from_numpy(pm).cuda() for pm in perms]
    maxit, s = 100, 201
    ps = [sfk.params("sflsqr", ell=2, maxit=maxit, sketch="sparse_sign", s=s, zeta=8, seed=5000 + i,
                     noise_norm=P.noise_norm, eta=1.01, perm=pts[j])
          for j, (i, P) in enumerate(zip(sel, probs))]
    ctx = sfk.init_batch(As, None, bs, ps)
    sfk.iterate(ctx, maxit)
    for j, (i, P) in enumerate(zip(sel, probs)):
        k_i, stopped_i, brk = sfk.instance_status(ctx, j)
        S = sketches.SparseSign(P.m, s, 8, 5000 + i)
        tol = fgk.discrepancy_tol(1.01, P.noise_norm, np.linalg.norm(P.b))
        orc = fgk.sketched_flexible(P.A, P.b, S, maxit=maxit, ell=2, tol=tol)
        assert stopped_i and not brk and k_i == orc.k, (j, k_i, orc.k)
        x = sfk.instance_solution(ctx, j, P.n).cpu().numpy()
        rho, _ = sfk.instance_residual_norms(ctx, j, k_i)
        assert rel(x, orc.x) <= 1e-8, (j, rel(x, orc.x))
        assert np.all(np.abs(rho[:k_i] - orc.rho[:k_i]) <= 1e-8 * orc.rho[:k_i]), j
        _, Xp, _, _, _ = gpu_run(P, "sflsqr", "sparse_sign", s, maxit, seed=5000 + i,
                                 noise=P.noise_norm, eta=1.01, perm=perms[j], stepwise=False)
        assert Xp.shape[1] == k_i
        assert rel(x, Xp[:, -1]) <= 1e-10
        say(f"instance {i} side {P.N} nnz {P.A.nnz}: stop k = {k_i} (oracle {orc.k}), "
            f"rel err vs oracle {rel(x, orc.x):.1e}")
    sfk.destroy(ctx)
