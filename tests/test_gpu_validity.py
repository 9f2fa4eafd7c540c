"""What the GPU result satisfies at the full workload sizes beyond the horizon
where two correctly rounded runs of the method stop agreeing on x_k and rho_k
(there element-wise agreement with an independent oracle is not determined by
the arithmetic; test_rounding_sensitivity_horizon pins that on the CPU).

  * eq. (FGK) for the GPU's own basis and coefficients:
    A z_j = sum_i h_ij w_i and B w_j = sum_i t_ij p_i, to rounding, every j;
  * the basis itself where it is reproducible: on the 256^2 unmatched workload
    two oracle summation orders give the same w_j, z_j, H and T to ~1e-11
    through k = 50 although x_k and rho_k separate from k ~ 13, so the GPU's
    basis and coefficients are compared with the oracle's element-wise to 1e-8;
  * the small sketched problem, in the GPU's own terms: rho_k does not increase,
    rho_k is the sketched residual of the returned x_k, and no y gives a smaller
    sketched residual over the GPU's range(Z_k).  Past the horizon the sketched
    matrix has condition ~1e15 and |y_k| ~1e13, so forming x_k = Z_k y_k loses
    digits: the oracle itself misses both identities by up to ~1e-2 relative
    there.  The GPU must be as consistent as the oracle: within 10 times the
    larger deviation of two oracle runs that differ only in the summation
    order of the sparse products (each row's nonzeros in stored and in reversed
    order), up to the same k (and 1e-9 where that is smaller).  One order alone
    is no yardstick: on the 64^2 workload the two orders miss the minimum by
    5e-9 and 1.3e-6 at k = 26, by 2e-6 and 3e-4 at k = 28.
"""
import numpy as np
import pytest
import torch

from oracle import fgk
from paper_2605_22281_amd import inputs

from gpu_cases import oracle_sketch, rel, say

pytestmark = pytest.mark.gpu


def _gpu_basis(P, method, kind, s, K, seed, perm=None):
    from paper_2605_22281_amd import sfk
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B) if P.B is not None else None
    b = torch.from_numpy(np.ascontiguousarray(P.b)).cuda()
    pt = torch.from_numpy(perm).cuda() if perm is not None else None
    ctx = sfk.init(A, B, b, sfk.params(method, maxit=K, sketch=kind, s=s, seed=seed, perm=pt))
    W = [sfk.basis_vector(ctx, "w", 1).cpu().numpy()]
    for k in range(1, K + 1):
        done, stopped, st = sfk.iterate(ctx, 1)
        assert done == k and not stopped and st == sfk.OK
        W.append(sfk.basis_vector(ctx, "w", k + 1).cpu().numpy())
    Z = np.stack([sfk.basis_vector(ctx, "z", j).cpu().numpy() for j in range(1, K + 1)], axis=1)
    Pm = np.stack([sfk.basis_vector(ctx, "p", j).cpu().numpy() for j in range(1, K + 1)], axis=1)
    H, T = sfk.coefficients(ctx, K)
    X = np.stack([sfk.solution_at(ctx, j).cpu().numpy() for j in range(1, K + 1)], axis=1)
    rho, _ = sfk.residual_norms(ctx)
    return dict(W=np.stack(W, axis=1), Z=Z, P=Pm, H=H, T=T, X=X, rho=rho)


def _ls_consistency(P, S, method, Z, X, rho, K):
    """Per k: |rho_k - ||S(A x_k - b)|| / that, and (rho_k - min_y ||M_k y - s||) / min,
    with M_k = S A Z_k (sFLSQR) or S B A Z_k (sFLSMR) formed on the host and the
    minimum from a Householder QR."""
    Bm = P.backprojector()
    SB = (lambda v: S.apply(Bm @ v)) if method == "sflsmr" else S.apply
    M = np.stack([SB(P.A @ Z[:, j]) for j in range(K)], axis=1)
    sb = SB(P.b)
    res, mn = [], []
    for k in range(1, K + 1):
        r = np.linalg.norm(SB(P.A @ X[:, k - 1] - P.b))
        res.append(abs(rho[k - 1] - r) / r)
        Q, _ = np.linalg.qr(M[:, :k])
        rmin = np.linalg.norm(sb - Q @ (Q.T @ sb))
        mn.append((rho[k - 1] - rmin) / rmin)
    return np.array(res), np.array(mn)


def _reversed_rows(M):
    """The same matrix with each row's nonzeros stored in reverse order."""
    R = M.tocsr().copy()
    for r in range(R.shape[0]):
        a, b = R.indptr[r], R.indptr[r + 1]
        R.indices[a:b] = R.indices[a:b][::-1].copy()
        R.data[a:b] = R.data[a:b][::-1].copy()
    R.has_sorted_indices = False
    return R


def _check(P, method, kind, s, K, seed, label, perm=None, basis_parity=0):
    g = _gpu_basis(P, method, kind, s, K, seed, perm)
    Bm = P.backprojector()
    S = oracle_sketch(method, kind, P, s, 8, seed)
    # eq. (FGK) for the GPU's own basis, column by column
    AZ = P.A @ g["Z"]
    fa = np.linalg.norm(AZ - g["W"] @ g["H"], axis=0) / np.linalg.norm(AZ, axis=0)
    BW = Bm @ g["W"][:, :K]
    fb = np.linalg.norm(BW - g["P"] @ g["T"], axis=0) / np.linalg.norm(BW, axis=0)
    say(f"{label}: eq. (FGK) worst column {fa.max():.1e} (A side) {fb.max():.1e} (B side)")
    assert fa.max() <= 1e-12 and fb.max() <= 1e-12
    assert np.allclose(np.linalg.norm(g["W"], axis=0), 1.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(g["P"], axis=0), 1.0, atol=1e-12)
    ii, jj = np.indices(g["H"].shape)
    assert np.all(g["H"][(ii < jj - 2) | (ii > jj + 1)] == 0)      # window ell = 2
    ii, jj = np.indices(g["T"].shape)
    assert np.all(g["T"][(ii < jj - 2) | (ii > jj)] == 0)
    # the oracle, for the basis comparison and as the consistency yardstick
    orc = fgk.sketched_flexible(P.A, P.b, S, method=method, B=P.B, maxit=K, ell=2)
    if basis_parity:
        kb = basis_parity
        ez = max(rel(g["Z"][:, j], orc.Z[:, j]) for j in range(kb))
        ew = max(rel(g["W"][:, j], orc.W[:, j]) for j in range(kb + 1))
        eh = np.max(np.abs(g["H"][:, :kb] - orc.H[:, :kb])) / np.max(np.abs(orc.H[:, :kb]))
        et = np.max(np.abs(g["T"][:kb, :kb] - orc.T[:kb, :kb])) / np.max(np.abs(orc.T[:kb, :kb]))
        say(f"{label}: basis vs oracle through k = {kb}: z {ez:.1e} w {ew:.1e} H {eh:.1e} T {et:.1e}")
        assert max(ez, ew, eh, et) <= 1e-8
    # the small problem
    rho = g["rho"]
    assert np.all(np.isfinite(g["X"])) and np.all(rho > 0)
    assert np.all(rho[1:] <= rho[:-1] * (1 + 1e-12))
    gres, gmin = _ls_consistency(P, S, method, g["Z"], g["X"], rho, K)
    ores, omin = _ls_consistency(P, S, method, orc.Z, orc.X, orc.rho, K)
    orv = fgk.sketched_flexible(_reversed_rows(P.A), P.b, S, method=method,
                                B=_reversed_rows(P.B) if P.B is not None else None, maxit=K, ell=2)
    ores2, omin2 = _ls_consistency(P, S, method, orv.Z, orv.X, orv.rho, K)
    ores = np.maximum(ores, ores2)
    omin = np.maximum(np.abs(omin), np.abs(omin2))
    # yardstick: the oracle's deviation up to k (running maximum over both orders)
    yres = np.maximum(1e-9, 10 * np.maximum.accumulate(ores))
    ymin = np.maximum(1e-9, 10 * np.maximum.accumulate(omin))
    say(f"{label}: rho vs ||S(A x - b)||: GPU worst {gres.max():.1e}, oracle worst {ores.max():.1e}; "
        f"rho above the minimum: GPU worst {gmin.max():.1e}, oracle {omin.max():.1e}")
    for k in range(K):
        assert gres[k] <= yres[k], (k + 1, gres[k], yres[k])
        assert gmin[k] <= ymin[k], (k + 1, gmin[k], ymin[k])


def test_ct64_fixed_50_validity():
    """64^2 CT, sFLSQR, sparse-sign s = 200, all 50 steps (x_k and rho_k are
    reproducible to 1e-8 through k ~ 22, the basis vectors through k ~ 10: two
    oracle summation orders differ by 7e-10 at k = 10 and 1e-8 at k = 11)."""
    P = inputs.workload("ct64")
    say("case: ct64 validity 50 steps")
    _check(P, "sflsqr", "sparse_sign", 200, 50, 3001, "ct64", basis_parity=10)


def test_ct256_unmatched_validity():
    """256^2 CT, unmatched B, sFLSMR with SRHT s = 400, 50 steps in the 4 x 4
    tile order bench.py uses: the basis and coefficients against the oracle
    through k = 50 (x_k and rho_k are reproducible through k ~ 12 only)."""
    P = inputs.workload("ct256_unmatched")
    say("case: ct256 validity 50 steps")
    _check(P, "sflsmr", "srht", 400, 50, 3002, "ct256", perm=inputs.tile_order(P.N, 4),
           basis_parity=50)
