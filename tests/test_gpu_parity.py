"""GPU parity: the HIP path (through the C ABI) against the CPU float64 oracle.

Bar: sketch indices and signs bit-exact; iterates x_k and minimised sketched
residual norms rho_k within 1e-8 relative while the problem is reproducible in
float64 (see gpu_cases.rounding_spread and the design notes).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import sketches
from paper_2605_22281_amd import inputs

from gpu_cases import compare, gpu_run, oracle_run, pinned, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ct24():
    return inputs.small_ct(24, 18, unmatched=True, noise=0.02)


@pytest.fixture(scope="module")
def ct24_sparse():
    return inputs.small_ct(24, 18, phantom="sparse", noise=0.01)


# ---------------------------------------------------------------- sketches

def test_sparse_sign_bit_exact():
    from paper_2605_22281_amd import sfk
    P = inputs.workload("ct64")
    say("case: sparse-sign sketch ct64 s=200 zeta=8")
    ctx, *_ = gpu_run(P, "sflsqr", "sparse_sign", 200, 3, seed=3001)
    rows, neg = sfk.sketch_sparse_sign(ctx)
    orc = sketches.SparseSign(P.m, 200, 8, 3001)
    assert np.array_equal(rows, orc.rows)
    assert np.array_equal(neg.astype(np.int64), (orc.signs < 0).astype(np.int64))


@pytest.mark.parametrize("method", ["sflsqr", "sflsmr"])
def test_srht_bit_exact(method):
    from paper_2605_22281_amd import sfk
    P = inputs.workload("ct64")       # m = 8190 pads to 8192, n = 4096 exact
    say(f"case: srht sketch ct64 {method}")
    ctx, *_ = gpu_run(P, method, "srht", 300, 3, seed=77)
    rows, neg = sfk.sketch_srht(ctx)
    d = P.m if method == "sflsqr" else P.n
    orc = sketches.SRHT(d, 300, 77)
    assert np.array_equal(rows, orc.rows)
    assert np.array_equal(neg.astype(bool), orc.D < 0)


def test_countsketch_and_instance_streams():
    from paper_2605_22281_amd import sfk
    P = inputs.small_ct(16, 12)
    say("case: countsketch instance 3")
    A = sfk.to_device_csr(P.A)
    import torch
    b = torch.from_numpy(P.b).cuda()
    ctx = sfk.init(A, None, b, sfk.params("sflsqr", s=40, maxit=5, sketch="countsketch", seed=9,
                                           instance=3))
    rows, neg = sfk.sketch_sparse_sign(ctx)
    orc = sketches.SparseSign(P.m, 40, 1, 9, instance=3)
    assert np.array_equal(rows, orc.rows)
    assert np.array_equal(neg.astype(np.int64), (orc.signs < 0).astype(np.int64))


# ---------------------------------------------------------------- small parity

SMALL_CASES = [
    # method, sketch, s, tau, ell, matched
    ("sflsqr", "sparse_sign", 60, "identity", 2, True),
    ("sflsqr", "sparse_sign", 60, "reweight_l1", 2, True),
    ("sflsqr", "srht", 60, "identity", 2, False),
    ("sflsmr", "srht", 60, "identity", 2, False),
    ("sflsmr", "sparse_sign", 60, "reweight_l1", 2, False),
    ("sflsqr", "sparse_sign", 60, "reweight_l1", 0, False),
    ("sflsqr", "sparse_sign", 60, "identity", 1, False),
    ("sflsmr", "srht", 60, "reweight_l1", 3, False),
    ("sflsqr", "countsketch", 60, "identity", 2, True),
]


@pytest.mark.parametrize("method,kind,s,tau,ell,matched", SMALL_CASES)
def test_parity_small_ct(ct24, method, kind, s, tau, ell, matched):
    P = ct24 if not matched else inputs.Problem(A=ct24.A, B=None, b=ct24.b, x_true=ct24.x_true,
                                                 noise_norm=ct24.noise_norm)
    maxit = 12
    say(f"case: small ct24 {method} {kind} tau={tau} ell={ell} matched={matched}")
    zeta = 1 if kind == "countsketch" else 8
    kind_o = "sparse_sign" if kind == "countsketch" else kind
    _, X, rho, _, st = gpu_run(P, method, kind, s, maxit, ell=ell, tau=tau, eps=1e-2, zeta=zeta)
    orc = oracle_run(P, method, kind_o, s, maxit, ell=ell, tau=tau, eps=1e-2, zeta=zeta)
    assert X.shape[1] == maxit
    compare(X, rho, orc, maxit, label=f"{method}/{kind}/{tau}/ell{ell}")


@pytest.mark.parametrize("method", ["sflsqr", "sflsmr"])
def test_parity_ragged_random(method):
    # empty rows, uneven row lengths, unmatched B, several workgroup tiles
    P = inputs.random_sparse_problem(3000, 1200, 0.004, seed=21, unmatched=True)
    say(f"case: random ragged 3000x1200 {method}")
    _, X, rho, _, _ = gpu_run(P, method, "sparse_sign", 120, 10, tau="reweight_l1", eps=0.1)
    orc = oracle_run(P, method, "sparse_sign", 120, 10, tau="reweight_l1", eps=0.1)
    compare(X, rho, orc, 10, label=f"ragged/{method}")


@pytest.mark.parametrize("vw", [-2, 0, 1, -1, 8, 16, 32, 64])
def test_parity_all_row_widths(ct24_sparse, vw):
    from paper_2605_22281_amd import sfk
    say(f"case: ct24 sparse vw={vw}")
    ctx, X, rho, _, _ = gpu_run(ct24_sparse, "sflsqr", "sparse_sign", 60, 8, tau="reweight_l1",
                                eps=1e-3, vw=vw)
    va, vb = sfk.spmv_variant(ctx)
    if vw >= 0:
        assert (va, vb) == (vw, vw)            # the requested kernel is the one that ran
    elif vw == -1:
        assert va in (8, 16, 32, 64) and vb in (8, 16, 32, 64)
    else:
        assert va in (0, 1) and vb in (0, 1)
    orc = oracle_run(ct24_sparse, "sflsqr", "sparse_sign", 60, 8, tau="reweight_l1", eps=1e-3)
    compare(X, rho, orc, 8, label=f"vw{vw}")


@pytest.mark.parametrize("vw", [0, 1, 64])
def test_parity_long_and_empty_rows(vw):
    # rows of up to 675 (A) and 1376 (B) nonzeros, i.e. several 512-nonzero
    # passes of the wave-per-row kernel, 125 empty rows, and the largest window
    # (ell = 8: with the full window the run stays reproducible in float64,
    # two summation orders of the oracle agree to 2e-13 through k = 9)
    from paper_2605_22281_amd import sfk
    P = inputs.random_sparse_problem(2000, 900, 0.7, seed=23, unmatched=True)
    say(f"case: long rows 2000x900 nnz={P.A.nnz} vw={vw}")
    ctx, X, rho, _, _ = gpu_run(P, "sflsmr", "sparse_sign", 120, 9, ell=8, vw=vw)
    assert sfk.spmv_variant(ctx) == (vw, vw)
    orc = oracle_run(P, "sflsmr", "sparse_sign", 120, 9, ell=8)
    compare(X, rho, orc, 9, label=f"long rows vw{vw}")


@pytest.mark.parametrize("vw", [0, 1])
def test_parity_wide_operator_32bit_columns(vw):
    # A with 70000 columns keeps 32-bit column indices in CSR-stream and
    # SELL-64; B (3000 columns) reads the 16-bit copies
    from paper_2605_22281_amd import sfk
    P = inputs.random_sparse_problem(3000, 70000, 0.0008, seed=29, unmatched=True)
    say(f"case: wide 3000x70000 nnz={P.A.nnz} vw={vw}")
    ctx, X, rho, _, _ = gpu_run(P, "sflsqr", "sparse_sign", 120, 8, vw=vw)
    assert sfk.spmv_variant(ctx)[0] == vw
    orc = oracle_run(P, "sflsqr", "sparse_sign", 120, 8)
    compare(X, rho, orc, 8, label=f"wide vw{vw}")


def test_identity_sketch_is_flsqr_type():
    # S = I (s = m): sFLSQR minimises the true residual over range(Z_k)
    P = inputs.small_ct(12, 10, n_det=17, unmatched=True)
    say(f"case: identity sketch m={P.m}")
    _, X, rho, _, _ = gpu_run(P, "sflsqr", "identity", P.m, 10, tau="reweight_l1", eps=0.05)
    orc = oracle_run(P, "sflsqr", "identity", P.m, 10, tau="reweight_l1", eps=0.05)
    compare(X, rho, orc, 10, label="identity-sketch")
    for k in range(10):
        assert abs(rho[k] - orc.res_true[k]) <= 1e-8 * orc.res_true[k]


# ---------------------------------------------------------------- the 64^2 workload

def test_ct64_discrepancy_run():
    """64x64 CT, 90 angles x 91 bins, sparse-sign s = 200, zeta = 8, maxit 50,
    discrepancy principle with eta = 1.01: same stopping iteration, all iterates."""
    P = inputs.workload("ct64")
    say("case: ct64 sFLSQR discrepancy")
    _, X, rho, rn, st = gpu_run(P, "sflsqr", "sparse_sign", 200, 50, noise=P.noise_norm, eta=1.01,
                                seed=3001)
    from oracle import fgk
    S = sketches.SparseSign(P.m, 200, 8, 3001)
    tol = fgk.discrepancy_tol(1.01, P.noise_norm, np.linalg.norm(P.b))
    orc = fgk.sketched_flexible(P.A, P.b, S, maxit=50, ell=2, tol=tol)
    assert orc.stopped and X.shape[1] == orc.k, (X.shape[1], orc.k)
    assert abs(rn - orc.rhs_norm) <= 1e-13 * orc.rhs_norm
    compare(X, rho, orc, orc.k, label="ct64-discrepancy")
    # the stop decision is not borderline
    thr = tol * orc.rhs_norm
    assert abs(orc.rho[-1] / thr - 1) > 1e-6


# ---------------------------------------------------------------- API semantics

def test_resume_equals_single_call_and_is_deterministic(ct24):
    from paper_2605_22281_amd import sfk
    say("case: resume/determinism")
    ctx1, *_ = gpu_run(ct24, "sflsmr", "srht", 60, 10, tau="reweight_l1", eps=1e-2, stepwise=False)
    x1 = sfk.solution(ctx1).cpu().numpy()
    ctx2, *_ = gpu_run(ct24, "sflsmr", "srht", 60, 10, tau="reweight_l1", eps=1e-2, stepwise=True,
                       **pinned(ctx1))
    x2 = sfk.solution(ctx2).cpu().numpy()
    assert np.array_equal(x1, x2)              # same launch sequence, fixed-order reductions
    r1, _ = sfk.residual_norms(ctx1)
    r2, _ = sfk.residual_norms(ctx2)
    assert np.array_equal(r1, r2)
    for j in (1, 5, 10):
        xa = sfk.solution_at(ctx1, j).cpu().numpy()
        xb = sfk.solution_at(ctx2, j).cpu().numpy()
        assert np.array_equal(xa, xb)
    with pytest.raises(sfk.SfkError):
        sfk.iterate(ctx1, 1)                   # capacity maxit exhausted


def test_happy_breakdown_identity_matrix():
    from paper_2605_22281_amd import sfk
    import torch
    n = 512
    say("case: A = I happy breakdown")
    A = sp.identity(n, format="csr")
    b = np.random.default_rng(3).standard_normal(n)
    P = inputs.Problem(A=inputs._as_int32_csr(A), B=None, b=b, x_true=b, noise_norm=0.0)
    ctx, X, rho, _, st = gpu_run(P, "sflsqr", "sparse_sign", 64, 10)
    assert st == sfk.BREAKDOWN and X.shape[1] == 1
    assert rel(X[:, 0], b) < 1e-14


def test_invalid_inputs_rejected():
    from paper_2605_22281_amd import sfk
    import torch
    say("case: invalid inputs")
    P = inputs.small_ct(16, 12)
    A = sfk.to_device_csr(P.A)
    p = sfk.params(s=40, maxit=5)
    with pytest.raises(sfk.SfkError) as e:
        sfk.init(A, None, torch.zeros(P.m, dtype=torch.float64, device="cuda"), p)
    assert e.value.status == sfk.EINVAL
    bad = sfk.to_device_csr(P.A)
    bad.colind[3] = P.n + 5
    with pytest.raises(sfk.SfkError) as e:
        sfk.init(bad, None, torch.from_numpy(P.b).cuda(), p)
    assert e.value.status == sfk.EINVAL
    nanb = torch.from_numpy(P.b).cuda()
    nanb[0] = float("nan")
    with pytest.raises(sfk.SfkError):
        sfk.init(A, None, nanb, p)


def test_true_residual_matches_host():
    from paper_2605_22281_amd import sfk
    P = inputs.small_ct(20, 16)
    say("case: true residual")
    ctx, X, *_ = gpu_run(P, "sflsqr", "sparse_sign", 50, 6)
    r = sfk.true_residual(ctx)
    assert abs(r - np.linalg.norm(P.b - P.A @ X[:, -1])) <= 1e-10 * r
