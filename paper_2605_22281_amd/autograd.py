"""torch.autograd.Function over the C ABI: x_K of K sFLSQR steps with the l1
reweighting, differentiable in the right-hand side b and the reweighting
parameter eps (the reverse sweep is the library's sfk_adjoint; this module
only marshals tensors)."""
from __future__ import annotations

import torch

from . import sfk


class SketchedFlexibleLSQR(torch.autograd.Function):
    """x = SketchedFlexibleLSQR.apply(b, eps, A, K, options)

    b: CUDA float64 tensor (m,) or (batch, m); eps: 0-dim CUDA or CPU float64
    tensor; A: sfk.DeviceCSR (m x n, B = A^T is built by the library); K:
    number of steps; options: dict of sfk.params keywords (sketch, s, zeta,
    seed, ell, tape, ...; instance r of a batch adds r to `instance`, so each
    right-hand side draws its own sketch stream).  Returns x_K with b's
    leading shape.  Backward gives dL/db and dL/deps (summed over the batch)."""

    @staticmethod
    def forward(ctx, b, eps, A, K, options):
        opts = dict(options or {})
        opts.setdefault("tape", 10)
        opts.setdefault("tau", "reweight_l1")
        e = float(eps.detach().cpu())
        rows = b.detach().reshape(-1, b.shape[-1]).contiguous()
        inst0 = int(opts.pop("instance", 0))
        ctxs, xs = [], []
        for r in range(rows.shape[0]):
            p = sfk.params("sflsqr", maxit=K, eps=e, instance=inst0 + r, **opts)
            c = sfk.init(A, None, rows[r].contiguous(), p)
            done, stopped, st = sfk.iterate(c, K)
            if done != K or stopped or st != sfk.OK:
                raise RuntimeError(f"right-hand side {r}: the run ended at step {done} of {K}")
            ctxs.append(c)
            xs.append(sfk.solution(c))
        ctx.sfk_contexts = ctxs
        ctx.b_shape = b.shape
        ctx.eps_device = eps.device
        x = torch.stack(xs)
        return x.reshape(*b.shape[:-1], A.cols)

    @staticmethod
    def backward(ctx, xbar):
        xb = xbar.detach().reshape(-1, xbar.shape[-1]).contiguous()
        bbars, ebar = [], 0.0
        for r, c in enumerate(ctx.sfk_contexts):
            bb, eb = sfk.adjoint(c, xb[r].contiguous())
            bbars.append(bb)
            ebar += eb
        for c in ctx.sfk_contexts:
            sfk.destroy(c)
        ctx.sfk_contexts = []
        bbar = torch.stack(bbars).reshape(ctx.b_shape)
        return bbar, torch.tensor(ebar, dtype=torch.float64, device=ctx.eps_device), None, None, None
