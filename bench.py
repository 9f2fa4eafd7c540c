#!/usr/bin/env python3
"""Throughput of the sketched flexible Golub-Kahan iteration on one MI355X.

Workload (default, the headline): sFLSQR with l1 reweighting on a 512 x 512
image (n = 262144), 360 angles x 725 bins (m = 261000), exact ray/pixel
intersection lengths A (1.2e8 nonzeros), B = A^T built on the device, sparse
phantom (2% of the pixels), 1% noise, sparse-sign sketch s = 600 (zeta = 8),
eps = 1e-3, FP64.  One step = one iteration of the method (forward projection,
truncated Gram-Schmidt, sketch, small sketched least squares, back-projection,
flexible preconditioner with the x assembly).  --steps K times the first K
iterations of a fresh context; the whole 300-iteration run is timed as well
(`full_run`, where the least-squares and x-assembly costs have grown with k).
Inputs are resident in HBM before every timed region; context set-up (init)
is outside them.

Beside the headline, in the same JSON line:
  * `workloads`: the 64^2 sFLSQR workload (50 iterations, and its discrepancy
    run) and the 256^2 unmatched sFLSMR workload (SRHT s = 400), each with its
    stage times and the roofline of its dominant product;
  * shared operator (`batched_multi_rhs`): R = 32 right-hand sides of the
    256^2 workload's A and B (own phantom, own SRHT seed each) in one context,
    against a loop of 32 plain solves on the same GPU; both run the same
    number of iterations, and every right-hand side's x_10 must agree with
    its plain run to 1e-8 relative;
  * heterogeneous (`batched_heterogeneous`): 32 independent instances, image
    side drawn from {128, 192, 256, 384} (angles 0.7 side, bins
    ceil(sqrt(2) side)), own ellipse phantom and noise U[0.5%, 3%], sFLSQR with
    B = A^T built on the device, sparse-sign s = 201, zeta = 8, up to 100
    iterations with the discrepancy principle per instance, against a plain
    loop over the same 32;
  * `deblur512`: the deblurring and inpainting workload (512^2 image, Gaussian
    blur of variance 0.25, 30% missing pixels, 5% noise, CountSketch s = 101,
    50 iterations) with the rank-30 truncation of every basis vector: FLSQR,
    sFLSQR, sFLSMR with the truncated SVD and the -RND variants with the
    randomized SVD, against plain sFLSQR;
  * `cpu_baseline`: the oracle on the headline workload, first iterations.

Prints one JSON line.  --gpus N with N > 1 is refused: this build runs on one
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sFLSQR iterations/sec + HBM GB/s (% peak); batched/plain speedup at 1e-8 rel"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "ct256_unmatched": dict(method="sflsmr", sketch="srht", s=400, zeta=8, iters=200, tau="identity",
                            seed=3002,
                            desc="256^2 CT (180 angles x 363 bins), unmatched pixel-driven B, "
                                 "sFLSMR, SRHT s=400, 200 iterations"),
    "ct64": dict(method="sflsqr", sketch="sparse_sign", s=200, zeta=8, iters=50, tau="identity",
                 seed=3001,
                 desc="64^2 CT (90 angles x 91 bins), B = A^T, sFLSQR, sparse-sign s=200 zeta=8, "
                      "50 iterations"),
    "ct512_sparse": dict(method="sflsqr", sketch="sparse_sign", s=600, zeta=8, iters=300,
                         tau="reweight_l1", seed=3003,
                         desc="512^2 CT (360 angles x 725 bins), B = A^T, sFLSQR with l1 "
                              "reweighting eps=1e-3, sparse-sign s=600 zeta=8, 300 iterations"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The sources of the single-instance SpMV kernels (k_spmv and what it includes):
# counter-derived traffic is only reported while these are unchanged.
SPMV_SOURCES = ("sfk_kernels.hip", "sfk_common.h", "sfk_dev.h", "sfk_sell.h", "sfk_beam.h")


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_22281_amd", "csrc")
    for f in SPMV_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def spmv_bytes(nnz: int, rows: int, cols: int, out_len: int, window: int,
               idx_bytes: int = 4) -> int:
    """Algorithmic bytes of one CSR SpMV launch with the fused window dots:
    8 B per nonzero value plus its column index (idx_bytes: 2 where the kernel
    reads the 16-bit copy), 4 B per row pointer, the gathered vector once, the
    output once, and the window vectors once."""
    return ((8 + idx_bytes) * nnz + 4 * (rows + 1) + 8 * cols + 8 * out_len
            + 8 * out_len * window)


def index_bytes(cols: int, kernel: str) -> int:
    """Bytes per column index read by the SpMV kernel: CSR-stream and SELL-64
    read 16-bit copies of operators with at most 65536 columns."""
    return 2 if cols <= 65536 and kernel in ("CSR-stream", "SELL-64") else 4


def copy_calibration(nbytes: int = 1 << 30):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))


def _timed_iterate(sfk, torch, ctx, k):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, stopped, st = sfk.iterate(ctx, k)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, done


def _order_tensor(order: str, P):
    """The order of the unknowns passed to the library (sfk_params.perm)."""
    import torch
    from paper_2605_22281_amd import inputs
    if order == "natural":
        return None
    return torch.from_numpy(inputs.tile_order(P.N, int(order[len("tiles"):]))).cuda()


def multi_rhs_bench(P, cfg, A, B, R: int, K: int, order: str = "natural"):
    """R right-hand sides sharing A and B in one context vs a loop of R plain
    solves, K iterations each (init outside the timed regions)."""
    import numpy as np
    import torch
    from paper_2605_22281_amd import inputs, sfk
    b, xt, _ = inputs.multi_rhs(P, R, seed=21)
    bb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    pt = _order_tensor(order, P)
    ps = [sfk.params(cfg["method"], ell=2, maxit=K, sketch=cfg["sketch"], s=cfg["s"],
                     zeta=cfg["zeta"], seed=3100 + r, tau=cfg["tau"], eps=1e-3, perm=pt)
          for r in range(R)]
    warm = sfk.init_multi(A, B, bb, ps)
    sfk.iterate(warm, min(K, 10))
    sfk.destroy(warm)
    ctx = sfk.init_multi(A, B, bb, ps)
    tb, done = _timed_iterate(sfk, torch, ctx, K)
    if done != K:
        raise SystemExit(f"shared-operator run ended after {done} of {K} iterations")
    kc = min(10, K)
    xb10 = [sfk.instance_solution_at(ctx, r, kc, P.n).cpu().numpy() for r in range(R)]
    xbK = [sfk.instance_solution(ctx, r, P.n).cpu().numpy() for r in range(R)]
    sfk.destroy(ctx)
    ctx = sfk.init_multi(A, B, bb, ps)
    sfk.set_timing(ctx, True)
    sfk.iterate(ctx, K)
    times = sfk.stage_times(ctx)
    sfk.destroy(ctx)
    tp, worst10, err_b, err_p = 0.0, 0.0, [], []
    for r in range(R):
        c = sfk.init(A, B, bb[r], ps[r])
        dt, d = _timed_iterate(sfk, torch, c, K)
        if d != K:
            raise SystemExit(f"plain run {r} ended after {d} of {K} iterations")
        tp += dt
        x10 = sfk.solution_at(c, kc).cpu().numpy()
        xK = sfk.solution(c).cpu().numpy()
        sfk.destroy(c)
        worst10 = max(worst10, float(np.linalg.norm(xb10[r] - x10) / np.linalg.norm(x10)))
        nt = np.linalg.norm(xt[r])
        err_b.append(float(np.linalg.norm(xbK[r] - xt[r]) / nt))
        err_p.append(float(np.linalg.norm(xK - xt[r]) / nt))
    rate_b, rate_p = R * K / tb, R * K / tp
    return {"R": R, "iterations": K, "workload": cfg["desc"] + f", {R} right-hand sides",
            "rhs_iterations_per_s": rate_b, "plain_rhs_iterations_per_s": rate_p,
            "speedup": rate_b / rate_p, "ms_per_batched_step": tb * 1e3 / K,
            "max_rel_diff_x10_vs_plain": worst10,
            "mean_rel_error_vs_truth": {"batched": float(np.mean(err_b)),
                                        "plain": float(np.mean(err_p))},
            "max_abs_diff_rel_error_vs_truth": float(np.max(np.abs(np.array(err_b) - np.array(err_p)))),
            "stage_avg_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in times.items()}}


def driver_compare(P, A, B, b, cfg, K, order):
    """The same K iterations with the stream driver and with each batch of
    iterations captured into a HIP graph (bit-identical results)."""
    import numpy as np
    import torch
    from paper_2605_22281_amd import sfk
    out = {}
    xs = {}
    vw = None           # the first context's SpMV kernels, repeated by every other
    for drv in ("multi", "graph"):
        kw = dict(vw=vw[0], vw_b=vw[1]) if vw else {}
        p = sfk.params(cfg["method"], ell=2, maxit=K, sketch=cfg["sketch"], s=cfg["s"],
                       zeta=cfg["zeta"], seed=cfg["seed"], tau=cfg["tau"], eps=1e-3, driver=drv,
                       perm=_order_tensor(order, P), **kw)
        if vw is None:
            ctx = sfk.init(A, B, b, p)
            vw = sfk.spmv_variant(ctx)
            sfk.destroy(ctx)
            p = sfk.params(cfg["method"], ell=2, maxit=K, sketch=cfg["sketch"], s=cfg["s"],
                           zeta=cfg["zeta"], seed=cfg["seed"], tau=cfg["tau"], eps=1e-3,
                           driver=drv, perm=_order_tensor(order, P), vw=vw[0], vw_b=vw[1])
        best = None
        for rep_ in range(3):
            ctx = sfk.init(A, B, b, p)
            dt, done = _timed_iterate(sfk, torch, ctx, K)
            xs[drv] = sfk.solution(ctx).cpu().numpy()
            sfk.destroy(ctx)
            best = dt if best is None else min(best, dt)
        out[drv] = {"iterations_per_s": K / best, "ms_per_step": best * 1e3 / K}
    out["bit_identical"] = bool(np.array_equal(xs["multi"], xs["graph"]))
    out["spmv_kernel"] = {"A": KERNEL_NAMES.get(vw[0], str(vw[0])), "B": KERNEL_NAMES.get(vw[1], str(vw[1]))}
    out["note"] = ("best of 3 runs of K iterations each, fresh context per run, the SpMV kernels "
                   "of the first context's tuner repeated in every context")
    return out


def full_vs_sketched(P, A, B, b, cfg, K, order):
    """Per-iteration time of the full-orthogonalisation method (FLSQR / FLSMR,
    Sec. 2.2) against the sketched one on the same operators, K iterations
    each (the paper's comparison of Sec. 3.2)."""
    import torch
    from paper_2605_22281_amd import sfk
    full = {"sflsqr": "flsqr", "sflsmr": "flsmr"}[cfg["method"]]
    res = {}
    for meth in (cfg["method"], full):
        p = sfk.params(meth, ell=2, maxit=K, sketch=cfg["sketch"], s=cfg["s"], zeta=cfg["zeta"],
                       seed=cfg["seed"], tau=cfg["tau"], eps=1e-3,
                       perm=_order_tensor(order, P) if meth == cfg["method"] else None)
        ctx = sfk.init(A, B, b, p)
        dt, done = _timed_iterate(sfk, torch, ctx, K)
        sfk.destroy(ctx)
        res[meth] = {"iterations": done, "iterations_per_s": done / dt, "ms_per_step": dt * 1e3 / done}
    res["sketched_speedup"] = res[cfg["method"]]["iterations_per_s"] / res[full]["iterations_per_s"]
    return res


def adjoint_bench(P, A, R=16, K=50, tape=10):
    """Forward (K reweighted sFLSQR steps with checkpoints every `tape`) and
    reverse sweep for R right-hand sides of the 256^2 operator with B = A^T
    (the differentiation workload), through the autograd.Function."""
    import numpy as np
    import torch
    from paper_2605_22281_amd import inputs
    from paper_2605_22281_amd.autograd import SketchedFlexibleLSQR
    bnp, xtnp, _ = inputs.multi_rhs(P, R, seed=31)
    b = torch.from_numpy(np.ascontiguousarray(bnp)).cuda().requires_grad_(True)
    eps = torch.tensor(1e-3, dtype=torch.float64, requires_grad=True)
    xt = torch.from_numpy(np.ascontiguousarray(xtnp)).cuda()
    opts = dict(sketch="srht", s=400, seed=3005, tape=tape)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = SketchedFlexibleLSQR.apply(b, eps, A, K, opts)
    loss = 0.5 * ((x - xt) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"rhs": R, "iterations": K, "checkpoint_every": tape,
            "forward_s": t1 - t0, "backward_s": t2 - t1,
            "note": "forward includes each right-hand side's init (B = A^T built on the device); "
                    "backward = reverse sweep with the basis regenerated between checkpoints",
            "grad_eps": float(eps.grad)}


def matrix_free_bench(P, name, K, W):
    """The workload with the operators computed on the fly (sfk_init_beam:
    exact Siddon projector and its exact transpose, or the interpolating
    back-projector when the workload's B is unmatched) instead of the stored
    matrices: K timed iterations, then the same with stage events."""
    import torch
    from paper_2605_22281_amd import sfk
    cfg = WORKLOADS[name]
    geo = sfk.BeamGeometry(P.N, P.n_angles, P.n_det, back=1 if P.B is not None else 0)
    b = torch.from_numpy(P.b).cuda()
    p = sfk.params(cfg["method"], ell=2, maxit=max(K, W, 1), sketch=cfg["sketch"], s=cfg["s"],
                   zeta=cfg["zeta"], seed=cfg["seed"], tau=cfg["tau"], eps=1e-3)
    if W > 0:
        c = sfk.init_beam(geo, b, p)
        sfk.iterate(c, W)
        sfk.destroy(c)
    c = sfk.init_beam(geo, b, p)
    dt, done = _timed_iterate(sfk, torch, c, K)
    sfk.destroy(c)
    c = sfk.init_beam(geo, b, p)
    sfk.set_timing(c, True)
    sfk.iterate(c, K)
    times = sfk.stage_times(c)
    sfk.destroy(c)
    return {"iterations": done, "iterations_per_s": done / dt, "ms_per_step": dt * 1e3 / done,
            "back_projector": "exact transpose" if geo.back == 0 else "pixel-driven interpolation",
            "stage_avg_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in times.items()}}


DEBLUR_METHODS = [
    # (label, method, tau, power iterations of the randomized SVD)
    ("sFLSQR (tau = I)", "sflsqr", "identity", 1),
    ("FLSQR tau_r", "flsqr", "lowrank", 1),
    ("sFLSQR tau_r", "sflsqr", "lowrank", 1),
    ("sFLSMR tau_r", "sflsmr", "lowrank", 1),
    ("sFLSQR-RND", "sflsqr", "lowrank_rnd", 1),
    ("sFLSMR-RND", "sflsmr", "lowrank_rnd", 1),
]


def deblur_bench(K: int = 50, r: int = 30, W: int = 2):
    """The deblurring and inpainting workload of the paper's timing comparison:
    512^2 image, Gaussian blur of variance 0.25 then 30% of the pixels missing,
    5% noise, CountSketch s = 101, rank r = 30 truncation of every basis vector
    (truncated SVD to a Ritz-residual tolerance of 1e-13, or the randomized SVD
    with 10 oversampling vectors and one power iteration), K = 50 iterations.
    Each method: W untimed warm-up iterations on a throw-away context, then K
    timed iterations of a fresh one, then the same K with stage events; and
    the relative error of x_K to the true image."""
    import numpy as np
    import torch
    from paper_2605_22281_amd import inputs, sfk
    P = inputs.workload("deblur512")
    A = sfk.to_device_csr(P.A)
    b = torch.from_numpy(P.b).cuda()
    xt = P.x_true
    out = {"workload": "512^2 Gaussian blur (variance 0.25) + 30% missing pixels + 5% noise, "
                       f"CountSketch s=101, rank {r}, {K} iterations",
           "m": P.m, "n": P.n, "nnz_A": int(P.A.nnz), "methods": {}}
    for label, method, tau, q in DEBLUR_METHODS:
        kw = dict(ell=2, maxit=K, sketch="sparse_sign", s=101, zeta=1, seed=3008, tau=tau,
                  lr_rows=P.N, lr_rank=r, lr_q=q)
        if W > 0:
            c = sfk.init(A, None, b, sfk.params(method, **{**kw, "maxit": max(W, 1)}))
            sfk.iterate(c, W)
            sfk.destroy(c)
        c = sfk.init(A, None, b, sfk.params(method, **kw))
        dt, done = _timed_iterate(sfk, torch, c, K)
        x = sfk.solution(c).cpu().numpy()
        stats = sfk.tau_stats(c) if tau.startswith("lowrank") else None
        sfk.destroy(c)
        c = sfk.init(A, None, b, sfk.params(method, **kw))
        sfk.set_timing(c, True)
        sfk.iterate(c, K)
        times = sfk.stage_times(c)
        sfk.destroy(c)
        res = {"iterations": done, "ms_total": dt * 1e3, "iterations_per_s": done / dt,
               "rel_error": float(np.linalg.norm(x - xt) / np.linalg.norm(xt)),
               "stage_ms_total": {k: v[0] for k, v in times.items() if v[1]}}
        if stats is not None:
            res["tau_last_call"] = stats
        out["methods"][label] = res
        log(f"bench: deblur512 {label}: {done} its in {dt * 1e3:.1f} ms, "
            f"error {res['rel_error']:.4f}")
    return out


def hetero_bench(count: int = 32, maxit: int = 100, order: str = "natural"):
    """Independent instances of uneven sizes in one context vs a plain loop."""
    import numpy as np
    import torch
    from paper_2605_22281_amd import inputs, sfk
    probs = inputs.batch_instances(count)
    As = [sfk.to_device_csr(P.A) for P in probs]       # separate device copies
    bs = [torch.from_numpy(np.ascontiguousarray(P.b)).cuda() for P in probs]
    perms = [_order_tensor(order, P) for P in probs]
    ps = [sfk.params("sflsqr", ell=2, maxit=maxit, sketch="sparse_sign", s=201, zeta=8,
                     seed=5000 + i, noise_norm=P.noise_norm, eta=1.01, perm=perms[i])
          for i, P in enumerate(probs)]
    warm = sfk.init_batch(As, None, bs, ps)
    sfk.iterate(warm, 5)
    sfk.destroy(warm)
    ctx = sfk.init_batch(As, None, bs, ps)
    tb, _ = _timed_iterate(sfk, torch, ctx, maxit)
    kb = [sfk.instance_status(ctx, i)[0] for i in range(count)]
    xb = [sfk.instance_solution(ctx, i, P.n).cpu().numpy() for i, P in enumerate(probs)]
    sfk.destroy(ctx)
    tp, kp, worst = 0.0, [], 0.0
    for i, P in enumerate(probs):
        c = sfk.init(As[i], None, bs[i], ps[i])
        dt, d = _timed_iterate(sfk, torch, c, maxit)
        tp += dt
        kp.append(d)
        x = sfk.solution(c).cpu().numpy()
        sfk.destroy(c)
        worst = max(worst, float(np.linalg.norm(xb[i] - x) / np.linalg.norm(x)))
    its = sum(kb)
    return {"instances": count, "sides": sorted({P.N for P in probs}),
            "nnz_total": int(sum(P.A.nnz for P in probs)), "maxit": maxit,
            "instance_iterations": its, "iterations_equal_plain": kb == kp,
            "instance_iterations_per_s": its / tb, "plain_instance_iterations_per_s": sum(kp) / tp,
            "speedup": (its / tb) / (sum(kp) / tp), "batched_s": tb, "plain_loop_s": tp,
            "max_rel_diff_x_vs_plain": worst}


def cpu_baseline(P, cfg, sample_iters: int):
    from oracle import fgk, sketches
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    d = P.m if cfg["method"] == "sflsqr" else P.n
    S = sketches.make(cfg["sketch"], d, cfg["s"], cfg["seed"], zeta=cfg["zeta"])
    B = P.B
    t0 = time.perf_counter()
    fgk.sketched_flexible(P.A, P.b, S, method=cfg["method"], B=B, maxit=sample_iters, ell=2,
                          tau=cfg["tau"], eps=1e-3)
    dt = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": sample_iters / dt, "unit": "iterations/s", "cores": blas_threads,
            "kind": "oracle",
            "sample": f"first {sample_iters} iterations of the same run "
                      f"({dt:.1f} s; scipy CSR products single-threaded, numpy BLAS "
                      f"{blas_threads} threads; {model}, {os.cpu_count()} logical CPUs)"}


KERNEL_NAMES = {0: "CSR-stream", 1: "SELL-64", 8: "8 lanes/row", 16: "16 lanes/row",
                32: "32 lanes/row", 64: "wave/row"}


def _load(name):
    import torch
    from paper_2605_22281_amd import inputs, sfk
    log(f"bench: generating {name}")
    t = time.perf_counter()
    P = inputs.workload(name)
    log(f"bench: {name}: m={P.m} n={P.n} nnzA={P.A.nnz} "
        f"nnzB={(P.B.nnz if P.B is not None else P.A.nnz)} ({time.perf_counter() - t:.1f} s)")
    dev = torch.device("cuda:0")
    A = sfk.to_device_csr(P.A, dev)
    B = sfk.to_device_csr(P.B, dev) if P.B is not None else None
    b = torch.from_numpy(P.b).to(dev)
    return P, A, B, b


def run_plain(name, P, A, B, b, K, W, args, full_run=False, noise=False):
    """Plain single-instance throughput: W untimed warm-up iterations on a
    throw-away context, K timed iterations of a fresh context, then the same K
    iterations once more with HIP events around every stage kernel (same SpMV
    kernels as the timed run: the automatic choice is repeated by vw/vw_b) for
    the stage averages and the roofline of the dominant product.  full_run:
    also the workload's whole iteration count, timed on a fresh context.
    noise: the discrepancy principle (eta = 1.01) instead of a fixed count."""
    import torch
    from paper_2605_22281_amd import sfk
    cfg = WORKLOADS[name]
    iters = cfg["iters"]
    maxit = max(K, W, iters if (full_run or noise) else 1)
    kw = dict(ell=2, maxit=maxit, sketch=cfg["sketch"], s=cfg["s"], zeta=cfg["zeta"],
              seed=cfg["seed"], tau=cfg["tau"], eps=1e-3, driver=args.driver,
              perm=_order_tensor(args.order, P))
    if noise:
        kw.update(noise_norm=P.noise_norm, eta=1.01)
    p = sfk.params(cfg["method"], vw=args.vw, **kw)
    if W > 0:
        ctx = sfk.init(A, B, b, p)
        sfk.iterate(ctx, W)
        sfk.destroy(ctx)
    ctx = sfk.init(A, B, b, p)
    va, vb = sfk.spmv_variant(ctx)
    elapsed, done = _timed_iterate(sfk, torch, ctx, K if not noise else iters)
    sfk.destroy(ctx)
    log(f"bench: {name}: timed {done} iterations in {elapsed * 1e3:.2f} ms")
    if not noise and done != K:
        raise SystemExit(f"{name}: run ended after {done} of {K} iterations")
    res = {"workload": cfg["desc"], "m": P.m, "n": P.n, "nnz_A": int(P.A.nnz),
           "nnz_B": int(P.B.nnz if P.B is not None else P.A.nnz), "method": cfg["method"],
           "sketch": cfg["sketch"], "s": cfg["s"], "iterations_timed": done,
           "iterations_per_s": done / elapsed, "ms_per_step": elapsed * 1e3 / max(done, 1),
           "spmv_kernel": {"A": KERNEL_NAMES.get(va, str(va)), "B": KERNEL_NAMES.get(vb, str(vb))}}
    if noise:
        res["stopped_at"] = done
        return res
    if full_run and iters > K:
        ctx = sfk.init(A, B, b, sfk.params(cfg["method"], vw=va, vw_b=vb, **kw))
        et, dn = _timed_iterate(sfk, torch, ctx, iters)
        sfk.destroy(ctx)
        res["full_run"] = {"iterations": dn, "iterations_per_s": dn / et,
                           "ms_per_step": et * 1e3 / dn}
        log(f"bench: {name}: full run {dn} iterations, {dn / et:.1f} it/s")
    ctx = sfk.init(A, B, b, sfk.params(cfg["method"], vw=va, vw_b=vb, **kw))
    assert sfk.spmv_variant(ctx) == (va, vb)
    sfk.set_timing(ctx, True)
    sfk.iterate(ctx, K)
    times = sfk.stage_times(ctx)
    sfk.destroy(ctx)
    ell = 2
    kA, kB = res["spmv_kernel"]["A"], res["spmv_kernel"]["B"]
    per_launch = {
        "spmv_A": spmv_bytes(P.A.nnz, P.m, P.n, P.m, ell + 1, index_bytes(P.n, kA)),
        "spmv_B": spmv_bytes(res["nnz_B"], P.n, P.m, P.n, ell, index_bytes(P.m, kB)),
    }
    stage_avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in times.items()}
    dom = max(("spmv_A", "spmv_B"), key=lambda q: times[q][0])
    achieved = per_launch[dom] / (stage_avg[dom] * 1e-3) / 1e9
    variant = kA if dom == "spmv_A" else kB
    traffic = None
    tr_file = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tr_file):
        try:
            entries = json.load(open(tr_file))
            entries = entries if isinstance(entries, list) else [entries]
            for tr in entries:
                # counters taken on the same kernel sources, workload, order of the
                # unknowns and SpMV variant as this run
                if (tr.get("source_hash") == source_hash() and tr.get("workload") == name
                        and tr.get("order") == args.order
                        and tr.get("variant", {}).get(dom) == variant):
                    traffic = tr.get("bytes_per_launch", {}).get(dom)
        except (OSError, ValueError):
            traffic = None
    # the whole iteration: both products' algorithmic bytes, the vector stages
    # (window reads, update writes), and the x assembly of the reweighting
    # (8 n (k - 1) bytes at step k, averaged over the timed steps)
    xbytes = 8 * P.n * (K - 1) / 2 if cfg["tau"] == "reweight_l1" else 0
    iter_bytes = (per_launch["spmv_A"] + per_launch["spmv_B"]
                  + 8 * (P.m * (ell + 3) + P.n * (ell + 3)) + xbytes)
    res["roofline"] = {"bound": "hbm", "kernel": dom, "variant": variant, "achieved": achieved,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                       "traffic": traffic, "bytes_per_launch": per_launch[dom],
                       "avg_launch_ms": stage_avg[dom]}
    res["iteration_GBps"] = iter_bytes / (res["ms_per_step"] * 1e-3) / 1e9
    res["iteration_frac"] = res["iteration_GBps"] / HBM_PEAK_GBS
    res["stage_avg_ms"] = stage_avg
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ct512_sparse", choices=sorted(WORKLOADS))
    ap.add_argument("--driver", default="auto", choices=["auto", "multi", "graph"])
    ap.add_argument("--vw", type=int, default=-2,
                    help="SpMV kernel: -2 automatic, 0 CSR-stream, 1 SELL-64, 8..64 lanes per row")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=None)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--batched", default="multi", choices=["all", "multi", "hetero", "none"],
                    help="batched comparisons: right-hand sides sharing the operators (multi) "
                         "and/or the heterogeneous batch of independent instances (hetero, not "
                         "in the default run while a memory fault seen with the heterogeneous "
                         "batch at these sizes has no known cause)")
    ap.add_argument("--extras", default="all", choices=["all", "none"],
                    help="the other plain workloads beside the headline")
    ap.add_argument("--no-full-run", action="store_true")
    ap.add_argument("--adjoint", type=int, default=1, help="time the derivative workload (0/1)")
    ap.add_argument("--rhs", type=int, default=32)
    ap.add_argument("--deblur", type=int, default=1,
                    help="time the deblurring workload with the low-rank operators (0/1)")
    ap.add_argument("--order", default="tiles4", choices=["natural", "tiles4", "tiles8"],
                    help="order of the unknowns passed to the library: the image's row-major "
                         "pixels, or 4x4 / 8x8 pixel tiles (results are in row-major order "
                         "either way)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the benchmark measures one GPU "
              f"(a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    name = args.workload
    cfg = WORKLOADS[name]
    K = args.steps if args.steps is not None else cfg["iters"]
    if K < 1 or K >= cfg["s"]:
        raise SystemExit(f"--steps must be in [1, {cfg['s'] - 1}] for this workload")
    W = args.warmup
    P, A, B, b = _load(name)
    head = run_plain(name, P, A, B, b, K, W, args, full_run=not args.no_full_run)
    out = {
        "metric": METRIC,
        "value": head["iterations_per_s"],
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["desc"] + f" (timed: iterations 1..{K} of a fresh context)",
                   "m": P.m, "n": P.n, "nnz_A": head["nnz_A"], "nnz_B": head["nnz_B"],
                   "method": cfg["method"], "sketch": cfg["sketch"], "s": cfg["s"], "ell": 2,
                   "driver": args.driver, "spmv_kernel": head["spmv_kernel"], "order": args.order},
        "roofline": head["roofline"],
        "iteration_GBps": head["iteration_GBps"],
        "iteration_frac": head["iteration_frac"],
        "stage_avg_ms": head["stage_avg_ms"],
    }
    if "full_run" in head:
        out["full_run"] = head["full_run"]
    if args.extras == "all":
        log("bench: matrix-free operators on the headline workload")
        out["matrix_free"] = matrix_free_bench(P, name, K, W)
    if not args.no_cpu_baseline:
        si = args.cpu_sample_iters or (12 if name == "ct512_sparse" else 40)
        log(f"bench: oracle baseline, {si} iterations")
        out["cpu_baseline"] = cpu_baseline(P, cfg, si)
    del A, B, b
    torch.cuda.empty_cache()
    others = [q for q in ("ct64", "ct256_unmatched", "ct512_sparse") if q != name]
    extras = {}
    keep = None
    for q in (others if args.extras == "all" else []):
        Pq, Aq, Bq, bq = _load(q)
        Kq = min(WORKLOADS[q]["iters"], WORKLOADS[q]["s"] - 1)
        extras[q] = run_plain(q, Pq, Aq, Bq, bq, Kq, W, args)
        if q == "ct64":
            extras[q]["discrepancy_run"] = run_plain(q, Pq, Aq, Bq, bq, Kq, 0, args, noise=True)
            extras[q]["drivers"] = driver_compare(Pq, Aq, Bq, bq, WORKLOADS[q], Kq, args.order)
        if q == "ct256_unmatched":
            keep = (Pq, Aq, Bq)
            extras[q]["full_vs_sketched"] = full_vs_sketched(Pq, Aq, Bq, bq, WORKLOADS[q], Kq,
                                                             args.order)
            if args.adjoint:
                log("bench: derivative workload (16 right-hand sides, 50 steps, forward + reverse)")
                extras["adjoint_ct256"] = adjoint_bench(Pq, Aq)
        else:
            del Aq, Bq, bq
    if extras:
        out["workloads"] = extras
    if args.batched in ("all", "multi"):
        q = "ct256_unmatched"
        if keep is None:
            Pq, Aq, Bq, _ = _load(q)
        else:
            Pq, Aq, Bq = keep
        Kq = min(K, WORKLOADS[q]["s"] - 1)
        log(f"bench: shared operator, {args.rhs} right-hand sides x {Kq} iterations, and plain loop")
        mr = multi_rhs_bench(Pq, WORKLOADS[q], Aq, Bq, args.rhs, Kq, args.order)
        out["batched_multi_rhs"] = mr
        out["batched_plain_speedup"] = mr["speedup"]
        log(f"bench: shared operator speedup {mr['speedup']:.2f}x")
    if args.extras == "all" and args.deblur:
        log("bench: deblurring workload with the low-rank operators")
        out["deblur512"] = deblur_bench()
    if args.batched in ("all", "hetero"):
        log("bench: heterogeneous batch of 32 instances, and plain loop")
        hb = hetero_bench(order=args.order)
        out["batched_heterogeneous"] = hb
        log(f"bench: heterogeneous speedup {hb['speedup']:.2f}x")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
