#!/usr/bin/env python3
"""Benchmark of the random-features-preconditioned KRR solve on one MI355X.

One step is the whole hot path on the multi-RHS workload (n = 65536 points, d = 54,
7 one-vs-all right-hand sides, s = 2048 random Fourier features, lambda = 1e-4 n, sigma
= median pairwise distance, tolerance 1e-6): random features, preconditioner
factorisation and mixed-precision PCG to 1e-6 (the three phases of Alg. 1), and the FP64
true residual at exit. Inputs are seeded synthetic data resident in HBM before timing.

Prints ONE JSON line. `value` is the whole-job kernel-product throughput: algorithmic
kernel-product flops 2 n^2 (d + m) of all products in the timed steps divided by the
timed wall time. `roofline` describes the dominant kernel (the fused kernel product) against
the dense FP16 MFMA peak: algorithmic flops per launch over the average launch time, timed with
HIP events inside the library on the stream it runs on; the executed MFMA work (split
products over padded widths) is reported beside it. `batched` is the solve of 64 uneven
problems in one plan (persistent product, captured iteration graph). `fp64_path` is the
same solve with the plain FP64 kernel product (time to tolerance), measured once after
the timed steps. `cpu_baseline` times the CPU FP64 oracle's kernel product on a row
sample on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts used by the roofline model
PEAK_MFMA_F16 = 2.5e15          # dense FP16/BF16 MFMA flop/s
PEAK_HBM = 8.0e12               # bytes/s
CUS, CLOCK = 256, 2.4e9
PEAK_EXP = CUS * 32 * CLOCK     # FP32 exp2 per second: 32 lanes per clock per CU


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536, help="points (65536 is the benchmark workload)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-problems solve")
    ap.add_argument("--extra", action="append", default=[], choices=["pixels", "differentiation"],
                    help="also run a full-size leg of another workload (repeatable)")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="run a plain device copy of this many bytes (counter calibration)")
    return ap.parse_args()


def source_sha256(rel):
    """Digest of a source file's code: comments and white space removed, so that editing a
    comment does not invalidate counters taken on the same kernels."""
    import hashlib
    import re
    with open(os.path.join(ROOT, rel)) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()


def recorded_traffic(kernel_src):
    """HBM bytes per launch of the kernel product from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_matmat_f16pv_mixture_n65536.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != source_sha256(kernel_src):
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def batched_run(dev):
    """The batched workload: 64 independent problems (n log-uniform in [1024, 16384], d in
    {16, 32, 64, 128}, s = n/8, 1-4 right-hand sides) solved to 1e-6 together."""
    import numpy as np
    import torch
    from paper_1611_03220_amd import krr
    from paper_1611_03220_amd import workloads as WL
    ws = WL.batched_instances()
    t0 = time.perf_counter()
    probs = []
    for w in ws:
        X = torch.from_numpy(w.X).to(dev)
        Z = krr.features(X, torch.from_numpy(w.W).to(dev), torch.from_numpy(w.b).to(dev))
        _, Ut = krr.precond_factor(Z, w.lam)
        del Z
        probs.append({"X": X, "sigma": w.sigma, "lam": w.lam, "Ut": Ut,
                      "Y": torch.from_numpy(np.ascontiguousarray(w.Y)).to(dev)})
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan = krr.BatchPlan(probs, tol=1e-6, refine=4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _, rep = plan.solve(raise_on_error=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    flops = sum(2.0 * w.n * w.n * (w.d + w.m) for w in ws)
    out = {"workload": "64 uneven problems, n in [1024, 16384], d in {16,32,64,128}, s = n/8",
           "status": rep.status, "time_to_tol_s": t3 - t2, "setup_features_factor_s": t1 - t0,
           "plan_create_s": t2 - t1, "iterations": rep.iters, "refine_steps": rep.refine_steps,
           "relres_true_max": max(max(r) for r in rep.relres_true),
           "product_ms": rep.product_ms, "iteration_ms": rep.iteration_ms,
           "product_tflops_algorithmic": flops / (rep.product_ms * 1e-3) / 1e12,
           "tiles_per_item": rep.tiles_per_item, "work_items": rep.work_items,
           "sum_n": int(sum(w.n for w in ws))}
    plan.close()
    return out


def _sync_time():
    import torch
    torch.cuda.synchronize()
    return time.perf_counter()


def pixels_run(dev):
    """Large dense-feature workload: n = 262144 pixel-like points (d = 784, 80 % zeros),
    10 one-vs-all right-hand sides, s = 8192 features, lambda = 1e-5 n, solved to 1e-6 with
    the mixed product and FP64-residual refinement."""
    import numpy as np
    import torch
    from paper_1611_03220_amd import krr
    from paper_1611_03220_amd import workloads as WL
    w = WL.pixels()
    X = torch.from_numpy(w.X).to(dev)
    Y = torch.from_numpy(np.ascontiguousarray(w.Y)).to(dev)
    W = torch.from_numpy(w.W).to(dev)
    b = torch.from_numpy(w.b).to(dev)
    t0 = _sync_time()
    Z = krr.features(X, W, b)
    t1 = _sync_time()
    _, Ut = krr.precond_factor(Z, w.lam)
    del Z
    t2 = _sync_time()
    _, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=w.tol, refine=3, raise_on_error=False)
    t3 = _sync_time()
    flops = 2.0 * w.n * w.n * (w.d + w.m)
    return {"workload": f"pixels n={w.n} d={w.d} m={w.m} s={w.s}", "status": rep.status,
            "time_to_tol_s": t3 - t0, "features_s": t1 - t0, "factor_s": t2 - t1,
            "solve_s": t3 - t2, "iterations": rep.iters, "refine_steps": rep.refine_steps,
            "relres_true_max": max(rep.relres_true), "matmat_calls": rep.matmat_calls,
            "matmat_tflops_algorithmic": flops * rep.matmat_calls / max(rep.matmat_ms, 1e-9) * 1e-9}


def differentiation_run(dev):
    """Differentiation workload: n = 131072 training + 16384 validation points, d = 440,
    147 one-vs-all columns, s = 4096; validation loss and its sigma / lambda gradients
    through the adjoint solve (mixed solves, FP64 derivative products)."""
    import numpy as np
    import torch
    from paper_1611_03220_amd import krr
    from paper_1611_03220_amd import autograd as KA
    from paper_1611_03220_amd import workloads as WL
    w = WL.correlated_differentiation()
    Xtr, Xv = torch.from_numpy(w.X).to(dev), torch.from_numpy(w.Xv).to(dev)
    Ytr = torch.from_numpy(np.ascontiguousarray(w.Y)).to(dev)
    Yv = torch.from_numpy(np.ascontiguousarray(w.Yv)).to(dev)
    t0 = _sync_time()
    Z = krr.features(Xtr, torch.from_numpy(w.W).to(dev), torch.from_numpy(w.b).to(dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    del Z
    t1 = _sync_time()
    sig = torch.tensor(w.sigma, dtype=torch.float64, device=dev, requires_grad=True)
    lam = torch.tensor(w.lam, dtype=torch.float64, device=dev, requires_grad=True)
    L = KA.validation_loss(Xtr, Ytr, Xv, Yv, sig, lam, Ut, tol=1e-6, refine=3)
    t2 = _sync_time()
    L.backward()
    t3 = _sync_time()
    return {"workload": f"differentiation n={w.n}+{w.Xv.shape[0]} d={w.d} m={w.m} s={w.s}",
            "setup_s": t1 - t0, "forward_s": t2 - t1, "backward_s": t3 - t2,
            "loss": float(L.detach()), "dL_dsigma": float(sig.grad), "dL_dlambda": float(lam.grad)}


def cpu_baseline(w, seconds):
    """Time the oracle's FP64 kernel product on a growing row sample for ~`seconds`."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    V = np.random.default_rng(0).standard_normal((w.n, w.m))
    rows_done, t_used, rows = 0, 0.0, 8
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        while t_used < seconds:
            idx = np.arange(rows_done, rows_done + rows) % w.n
            t0 = time.perf_counter()
            O.kernel_matmat(w.X, w.X, w.sigma, V, rows=idx)
            t_used += time.perf_counter() - t0
            rows_done += rows
            rows = min(rows * 2, 256)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    flops = 2.0 * rows_done * w.n * (w.d + w.m)
    return {"value": flops / t_used / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 difference-form kernel product K[rows, :] V for {rows_done} of "
                      f"{w.n} rows (d={w.d}, m={w.m}), {t_used:.1f} s, one thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is single-GPU "
              "by design; the design notes describe how it would shard", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1611_03220_amd import krr
    from paper_1611_03220_amd import workloads as WL

    dev = torch.device("cuda:0")
    w = WL.mixture_multi_rhs(n=args.n)
    X = torch.from_numpy(w.X).to(dev)
    Y = torch.from_numpy(np.ascontiguousarray(w.Y)).to(dev)
    W = torch.from_numpy(w.W).to(dev)
    b = torch.from_numpy(w.b).to(dev)
    torch.cuda.synchronize()
    if args.calib_bytes > 0:
        # a plain copy kernel of known size: what the byte counters read for it calibrates
        # the counters of the kernels profiled in the same run
        src = torch.ones(args.calib_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def step(prec):
        Z = krr.features(X, W, b)
        _, Ut = krr.precond_factor(Z, w.lam)
        alpha, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=w.tol, prec=prec,
                                   true_residual=True, raise_on_error=False)
        return alpha, rep

    for _ in range(args.warmup):
        step("f16x3")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [step("f16x3")[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    n, d, m = w.n, w.d, w.m
    flops_mm = 2.0 * n * n * (d + m)
    calls = sum(r.matmat_calls for r in reps)
    mm_ms = sum(r.matmat_ms for r in reps)
    avg_launch_s = mm_ms / max(calls, 1) / 1e3
    pairs = float(n) * n
    kp = int(math.ceil((d + 2) / 32.0) * 32)        # augmented, padded feature width
    mp = int(math.ceil(m / 16.0) * 16)              # padded right-hand-side columns
    # split-3 distances; P V takes three split products, or two when m <= 8 (the hi and lo
    # parts of V share one 16-column operand)
    exec_mfma = pairs * 2 * (3 * kp + (2 if m <= 8 else 3) * mp)
    roof = {"bound": "mfma", "achieved": flops_mm / avg_launch_s / 1e12,
            "peak": PEAK_MFMA_F16 / 1e12, "unit": "TFLOP/s",
            "frac": flops_mm / avg_launch_s / PEAK_MFMA_F16,
            "traffic": recorded_traffic("paper_1611_03220_amd/csrc/matmat.hip"),
            "kernel": "matmat_f16pv_kernel (FP16 hi/lo split MFMA distances, FP32 exp2, "
                      "split MFMA accumulation of K V, FP64 partial sums)",
            "algorithmic_flops_per_launch": flops_mm, "avg_launch_ms": avg_launch_s * 1e3,
            "launches": calls,
            "executed_mfma_flops_per_launch": exec_mfma,
            "executed_mfma_tflops": exec_mfma / avg_launch_s / 1e12,
            "executed_frac": exec_mfma / avg_launch_s / PEAK_MFMA_F16,
            "exp_per_s": pairs / avg_launch_s, "exp_peak_per_s": PEAK_EXP,
            "exp_frac": pairs / avg_launch_s / PEAK_EXP,
            "timed_with": "HIP events on the library's stream around every product launch"}
    relres_true = max(max(r.relres_true) for r in reps)
    iters = [r.iters for r in reps]
    out = {
        "metric": "kernel matmat TFLOP/s + time-to-1e-6 residual PCG solve, mixed vs FP64 path",
        "value": calls * flops_mm / wall / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16x3-split MFMA + f32 exp, f64 CG scalars", "data": "synthetic",
        "config": {"workload": "multi-RHS Gaussian mixture", "n": n, "d": d, "m": m, "s": w.s,
                   "lambda": w.lam, "sigma": w.sigma, "tol": w.tol, "parallelism": "single GPU"},
        "time_to_tol_mixed_s": wall / args.steps,
        "iterations": iters,
        "relres_true_max": relres_true,
        "kernel_matmat_tflops": flops_mm / avg_launch_s / 1e12,
        "roofline": roof,
    }
    if not args.no_fp64:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, r64 = step("fp64")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        out["fp64_path"] = {"time_to_tol_s": t64, "iterations": r64.iters,
                            "relres_true_max": max(r64.relres_true),
                            "kernel_matmat_tflops": flops_mm * r64.matmat_calls / max(r64.matmat_ms, 1e-9) * 1e-9,
                            "speedup_mixed_vs_fp64": t64 / (wall / args.steps)}
        print(f"[bench] fp64 path {t64:.3f} s", file=sys.stderr, flush=True)
    if not args.no_batched:
        del X, Y, W, b
        torch.cuda.empty_cache()
        out["batched"] = batched_run(dev)
        print(f"[bench] batched solve {out['batched']['time_to_tol_s']:.3f} s", file=sys.stderr,
              flush=True)
    for extra in args.extra:
        torch.cuda.empty_cache()
        out[extra] = pixels_run(dev) if extra == "pixels" else differentiation_run(dev)
        print(f"[bench] {extra}: {out[extra]}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
