#!/usr/bin/env python3
"""Throughput of the sketched flexible Golub-Kahan iteration on one MI355X.

Workload (default): 256 x 256 image (n = 65536), 180 angles x 363 bins
(m = 65340), exact ray/pixel intersection lengths A, unmatched pixel-driven
back-projector B, ellipse phantom, 2% noise; sFLSMR with an SRHT sketch of
s = 400 rows, 200 iterations, FP64.  One step = one iteration of the method
(forward projection, truncated Gram-Schmidt, sketch, small sketched least
squares, back-projection, flexible preconditioner).  Inputs are resident in HBM
before the timed region; the context set-up (init) is outside it.

Batched throughput, reported beside the plain figure (same JSON line):
  * shared operator: R = 32 right-hand sides of the default workload's A and B
    (own phantom, own SRHT seed each) in one context, against a loop of 32
    plain solves on the same GPU; both run the same number of iterations, and
    every right-hand side's x_10 must agree with its plain run to 1e-8 relative;
  * heterogeneous: 32 independent instances, image side drawn from
    {128, 192, 256, 384} (angles 0.7 side, bins ceil(sqrt(2) side)), own
    ellipse phantom and noise U[0.5%, 3%], sFLSQR with B = A^T built on the
    device, sparse-sign s = 201, zeta = 8, up to 100 iterations with the
    discrepancy principle per instance, against a plain loop over the same 32.
Set-up (init) is outside every timed region.

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
                            desc="256^2 CT (180 angles x 363 bins), unmatched pixel-driven B, "
                                 "sFLSMR, SRHT s=400, 200 iterations"),
    "ct64": dict(method="sflsqr", sketch="sparse_sign", s=200, zeta=8, iters=50, tau="identity",
                 desc="64^2 CT (90 angles x 91 bins), B = A^T, sFLSQR, sparse-sign s=200 zeta=8, "
                      "50 iterations"),
    "ct512_sparse": dict(method="sflsqr", sketch="sparse_sign", s=600, zeta=8, iters=300,
                         tau="reweight_l1",
                         desc="512^2 CT (360 angles x 725 bins), B = A^T, sFLSQR with l1 "
                              "reweighting eps=1e-3, sparse-sign s=600 zeta=8, 300 iterations"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_22281_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
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
    S = sketches.make(cfg["sketch"], d, cfg["s"], 3000 + 2, zeta=cfg["zeta"])
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ct256_unmatched", choices=sorted(WORKLOADS))
    ap.add_argument("--driver", default="auto", choices=["auto", "multi", "persistent"])
    ap.add_argument("--vw", type=int, default=-2,
                    help="SpMV kernel: -2 automatic, 0 CSR-stream, 1 SELL-64, 8..64 lanes per row")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=40)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--batched", default="all", choices=["all", "multi", "hetero", "none"])
    ap.add_argument("--rhs", type=int, default=32)
    ap.add_argument("--order", default="tiles4", choices=["natural", "tiles4", "tiles8"],
                    help="order of the unknowns passed to the library: the image's row-major "
                         "pixels, or 4x4 / 8x8 pixel tiles (results are in row-major order "
                         "either way)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build measures one GPU "
              f"(a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch
    from paper_2605_22281_amd import inputs, sfk

    cfg = WORKLOADS[args.workload]
    K = args.steps if args.steps is not None else cfg["iters"]
    if K < 1 or K >= cfg["s"]:
        raise SystemExit(f"--steps must be in [1, {cfg['s'] - 1}] for this workload")
    W = args.warmup
    log(f"bench: generating {args.workload}")
    t = time.perf_counter()
    P = inputs.workload(args.workload)
    log(f"bench: m={P.m} n={P.n} nnzA={P.A.nnz} nnzB={(P.B.nnz if P.B is not None else P.A.nnz)} "
        f"({time.perf_counter() - t:.1f} s)")
    dev = torch.device("cuda:0")
    A = sfk.to_device_csr(P.A, dev)
    B = sfk.to_device_csr(P.B, dev) if P.B is not None else None
    b = torch.from_numpy(P.b).to(dev)
    maxit = max(K, W, 1)
    p = sfk.params(cfg["method"], ell=2, maxit=maxit, sketch=cfg["sketch"], s=cfg["s"],
                   zeta=cfg["zeta"], seed=3000 + 2, tau=cfg["tau"], eps=1e-3, driver=args.driver,
                   vw=args.vw, perm=_order_tensor(args.order, P))

    if W > 0:
        log(f"bench: warmup {W} iterations")
        ctx = sfk.init(A, B, b, p)
        sfk.iterate(ctx, W)
        sfk.destroy(ctx)

    # timed region: K iterations of a fresh context (init outside)
    ctx = sfk.init(A, B, b, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, stopped, st = sfk.iterate(ctx, K)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"bench: timed {done} iterations in {elapsed * 1e3:.2f} ms")
    if done != K:
        raise SystemExit(f"run ended after {done} of {K} iterations (status {st})")
    names = {0: "CSR-stream", 1: "SELL-64", 8: "8 lanes/row", 16: "16 lanes/row",
             32: "32 lanes/row", 64: "wave/row"}
    timed_kernel = {op: names.get(v, str(v)) for op, v in zip(("A", "B"), sfk.spmv_variant(ctx))}
    sfk.destroy(ctx)

    # same work again with HIP events around every stage kernel (library stream);
    # each init chooses its SpMV kernels by timing them, so both choices are kept
    ctx = sfk.init(A, B, b, p)
    spmv_kernel = {op: names.get(v, str(v)) for op, v in zip(("A", "B"), sfk.spmv_variant(ctx))}
    sfk.set_timing(ctx, True)
    sfk.iterate(ctx, K)
    times = sfk.stage_times(ctx)
    sfk.destroy(ctx)

    nnzA = P.A.nnz
    nnzB = P.B.nnz if P.B is not None else P.A.nnz
    ell = 2
    per_launch = {
        "spmv_A": spmv_bytes(nnzA, P.m, P.n, P.m, ell + 1, index_bytes(P.n, spmv_kernel["A"])),
        "spmv_B": spmv_bytes(nnzB, P.n, P.m, P.n, ell, index_bytes(P.m, spmv_kernel["B"])),
    }
    stage_avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in times.items()}
    dom = max(("spmv_A", "spmv_B"), key=lambda s: times[s][0])
    achieved = per_launch[dom] / (stage_avg[dom] * 1e-3) / 1e9
    traffic = None
    tr_file = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tr_file):
        try:
            tr = json.load(open(tr_file))
            # counters taken on the same kernel sources, workload, order of the
            # unknowns and SpMV variant as this run
            op = "A" if dom == "spmv_A" else "B"
            if (tr.get("source_hash") == source_hash() and tr.get("workload") == args.workload
                    and tr.get("order") == args.order
                    and tr.get("variant", {}).get(dom) == spmv_kernel[op]):
                traffic = tr.get("bytes_per_launch", {}).get(dom)
        except (OSError, ValueError):
            traffic = None

    ms_per_step = elapsed * 1e3 / K
    iter_bytes = per_launch["spmv_A"] + per_launch["spmv_B"] + 8 * (P.m * (ell + 3) + P.n * (ell + 3))
    out = {
        "metric": METRIC,
        "value": K / elapsed,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "m": P.m, "n": P.n, "nnz_A": nnzA, "nnz_B": nnzB,
                   "method": cfg["method"], "sketch": cfg["sketch"], "s": cfg["s"], "ell": ell,
                   "driver": args.driver, "spmv_kernel": timed_kernel, "order": args.order},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "variant": spmv_kernel["A" if dom == "spmv_A" else "B"],
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": per_launch[dom], "avg_launch_ms": stage_avg[dom]},
        "iteration_GBps": iter_bytes / (ms_per_step * 1e-3) / 1e9,
        "stage_avg_ms": stage_avg,
    }
    if args.batched in ("all", "multi"):
        log(f"bench: shared operator, {args.rhs} right-hand sides x {K} iterations, and plain loop")
        mr = multi_rhs_bench(P, cfg, A, B, args.rhs, K, args.order)
        out["batched_multi_rhs"] = mr
        out["batched_plain_speedup"] = mr["speedup"]
        log(f"bench: shared operator speedup {mr['speedup']:.2f}x")
    if args.batched in ("all", "hetero"):
        log("bench: heterogeneous batch of 32 instances, and plain loop")
        hb = hetero_bench(order=args.order)
        out["batched_heterogeneous"] = hb
        log(f"bench: heterogeneous speedup {hb['speedup']:.2f}x")
    if not args.no_cpu_baseline:
        log(f"bench: oracle baseline, {args.cpu_sample_iters} iterations")
        out["cpu_baseline"] = cpu_baseline(P, cfg, args.cpu_sample_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
