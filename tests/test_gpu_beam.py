"""Matrix-free parallel-beam operators (sfk_init_beam) against the explicit
matrices the host generator builds for the same geometry (the Siddon
intersection lengths and the pixel-driven interpolating back-projector), and
the method with them against the oracle run on those matrices."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import fgk, sketches
from paper_2605_22281_amd import inputs

from gpu_cases import compare, rel, say

pytestmark = pytest.mark.gpu


def _ctx(geo, b_np, p):
    from paper_2605_22281_amd import sfk
    b = torch.from_numpy(np.ascontiguousarray(b_np)).cuda()
    return sfk.init_beam(geo, b, p)


@pytest.mark.parametrize("N,na,nd,nz", [(16, 12, 23, 1), (24, 18, 34, 1), (15, 10, 22, 1),
                                        (12, 8, 17, 3), (64, 90, 91, 1)])
def test_operators_match_the_stored_matrices(N, na, nd, nz):
    from paper_2605_22281_amd import sfk
    say(f"case: beam operators N={N} na={na} nd={nd} nz={nz}")
    A2 = inputs.siddon_matrix(N, na, nd)
    Bp2 = inputs.pixel_driven_backprojector(N, na, nd)
    A = sp.block_diag([A2] * nz, format="csr")
    Bp = sp.block_diag([Bp2] * nz, format="csr")
    rng = np.random.default_rng(N + nz)
    x = rng.standard_normal(A.shape[1])
    w = rng.standard_normal(A.shape[0])
    for back, Bm in ((0, A.T.tocsr()), (1, Bp)):
        geo = sfk.BeamGeometry(N, na, nd, nz=nz, back=back)
        ctx = _ctx(geo, A @ rng.random(A.shape[1]), sfk.params("sflsqr", maxit=2, s=min(40, A.shape[0] - 1)))
        y = sfk.apply(ctx, "A", torch.from_numpy(x).cuda()).cpu().numpy()
        z = sfk.apply(ctx, "B", torch.from_numpy(w).cuda()).cpu().numpy()
        assert np.linalg.norm(y - A @ x) <= 1e-13 * np.linalg.norm(A @ x)
        assert np.linalg.norm(z - Bm @ w) <= 1e-13 * np.linalg.norm(Bm @ w)
        # per-ray and per-pixel agreement (the same pieces, summed in another order)
        assert np.max(np.abs(y - A @ x)) <= 1e-12 * np.max(np.abs(A @ x))
        assert np.max(np.abs(z - Bm @ w)) <= 1e-12 * np.max(np.abs(Bm @ w))


@pytest.mark.parametrize("method,kind,back,tau", [("sflsqr", "sparse_sign", 0, "reweight_l1"),
                                                  ("sflsmr", "srht", 1, "identity"),
                                                  ("flsqr", None, 0, "reweight_l1")])
def test_method_with_beam_operators_against_oracle(method, kind, back, tau):
    from paper_2605_22281_amd import sfk
    P = inputs.small_ct(24, 18, unmatched=(back == 1), noise=0.02)
    say(f"case: beam {method} back={back} tau={tau}")
    geo = sfk.BeamGeometry(P.N, P.n_angles, P.n_det, back=back)
    k = 12
    if method == "flsqr":
        p = sfk.params("flsqr", maxit=k, tau=tau, eps=1e-2)
        orc = fgk.flexible_full(P.A, P.b, method="flsqr", maxit=k, tau=tau, eps=1e-2)
    else:
        d = P.m if method == "sflsqr" else P.n
        p = sfk.params(method, maxit=k, sketch=kind, s=60, seed=9, tau=tau, eps=1e-2)
        S = sketches.make(kind, d, 60, 9)
        orc = fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=k, ell=2, tau=tau,
                                    eps=1e-2)
    ctx = _ctx(geo, P.b, p)
    done, _, _ = sfk.iterate(ctx, k)
    assert done == k
    X = np.stack([sfk.solution_at(ctx, j).cpu().numpy() for j in range(1, k + 1)], axis=1)
    rho, _ = sfk.residual_norms(ctx)
    compare(X, rho, orc, k, label=f"beam {method}")
    rt, _ = sfk.residual_norms(ctx, "true_explicit")
    assert np.max(np.abs(rt - orc.res_true) / orc.res_true) <= 1e-8


def test_ct512_reweighted_matrix_free():
    """512^2, 360 x 725: the reweighted sFLSQR workload with the operators
    computed on the fly, against the oracle on the stored matrix (k <= 20)."""
    from paper_2605_22281_amd import sfk
    P = inputs.workload("ct512_sparse")
    say("case: beam ct512 reweighted sFLSQR")
    geo = sfk.BeamGeometry(P.N, P.n_angles, P.n_det, back=0)
    k = 20
    ctx = _ctx(geo, P.b, sfk.params("sflsqr", maxit=k, sketch="sparse_sign", s=600, seed=3003,
                                    tau="reweight_l1", eps=1e-3))
    done, _, _ = sfk.iterate(ctx, k)
    X = np.stack([sfk.solution_at(ctx, j).cpu().numpy() for j in range(1, k + 1)], axis=1)
    rho, _ = sfk.residual_norms(ctx)
    S = sketches.SparseSign(P.m, 600, 8, 3003)
    orc = fgk.sketched_flexible(P.A, P.b, S, maxit=k, ell=2, tau="reweight_l1", eps=1e-3)
    compare(X, rho, orc, k, label="beam ct512")
