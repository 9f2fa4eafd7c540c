"""The allocation-free solve (sfk_solve_noalloc) against the context entry
points (sfk_init / sfk_iterate / sfk_solution) on the same inputs: two calls
in a row, the second on a smaller problem, and a problem too large for the
library's fixed scratch."""
import numpy as np
import pytest
import torch

from paper_2605_22281_amd import inputs, sfk

from gpu_cases import rel, say

pytestmark = pytest.mark.gpu


def _reference(P, p, k):
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B) if P.B is not None else None
    b = torch.from_numpy(np.ascontiguousarray(P.b)).cuda()
    ctx = sfk.init(A, B, b, p)
    done, stopped, _ = sfk.iterate(ctx, k)
    x = sfk.solution(ctx).cpu().numpy()
    rho, _ = sfk.residual_norms(ctx)
    sfk.destroy(ctx)
    return x, rho, done, stopped


def _noalloc(P, p, k):
    A = sfk.to_device_csr(P.A)
    B = sfk.to_device_csr(P.B) if P.B is not None else None
    b = torch.from_numpy(np.ascontiguousarray(P.b)).cuda()
    x, rho, done, stopped, st = sfk.solve_noalloc(A, B, b, p, k)
    torch.cuda.synchronize()
    return x.cpu().numpy(), rho, done, stopped


def test_noalloc_matches_context_two_calls():
    big = inputs.small_ct(32, 24, unmatched=True, noise=0.02, seed_offset=61)
    small = inputs.small_ct(16, 12, phantom="sparse", noise=0.01, seed_offset=62)
    cases = [
        (big, sfk.params("sflsmr", maxit=14, sketch="srht", s=80, seed=7, tau="reweight_l1",
                         eps=1e-2, vw=0, copies=1), 14),
        (small, sfk.params("sflsqr", maxit=9, sketch="sparse_sign", s=60, seed=8, vw=0,
                           copies=1), 9),
    ]
    for P, p, k in cases:
        say(f"case: noalloc m={P.m} n={P.n} method={p.method} k={k}")
        xr, rr, dr, sr = _reference(P, p, k)
        xn, rn, dn, sn = _noalloc(P, p, k)
        assert (dn, sn) == (dr, sr) == (k, False)
        ex, er = rel(xn, xr), np.max(np.abs(rn - rr) / rr)
        say(f"noalloc vs context: x {ex:.1e} rho {er:.1e}")
        assert ex <= 1e-8 and er <= 1e-8


def test_noalloc_discrepancy_stop_and_true_residual():
    P = inputs.small_ct(24, 18, noise=0.03, seed_offset=63)
    say("case: noalloc discrepancy stop")
    p = sfk.params("sflsqr", maxit=30, s=70, seed=9, noise_norm=P.noise_norm, eta=1.01, vw=0,
                   copies=1, resid=1)
    xr, rr, dr, sr = _reference(P, p, 30)
    xn, rn, dn, sn = _noalloc(P, p, 30)
    assert sr and sn and dn == dr < 30
    assert rel(xn, xr) <= 1e-8 and np.max(np.abs(rn - rr) / rr) <= 1e-8


def test_noalloc_rejects_too_large_before_device_work():
    A = sfk.host_csr_descriptor(261000, 262144, 120155712)
    p = sfk.params("sflsqr", maxit=300, s=600)
    x = torch.empty(262144, dtype=torch.float64, device="cuda")
    rho = (sfk.ctypes.c_double * 300)()
    st = sfk.lib().sfk_solve_noalloc(sfk.ctypes.byref(A), None, None, sfk.ctypes.byref(p), 10,
                                     x.data_ptr(), rho, None, None, None)
    assert st == sfk.ENOMEM
    assert b"SFK_NOALLOC_BYTES" in sfk.lib().sfk_last_error(None)
    with pytest.raises(sfk.SfkError):
        Q = inputs.small_ct(12, 10)
        sfk.solve_noalloc(sfk.to_device_csr(Q.A), None, torch.from_numpy(Q.b).cuda(),
                          sfk.params("sflsqr", maxit=5, s=40, vw=1), 5)
