"""Benchmark: factor + solve throughput of random-multiplier GENP on one MI355X.

One step is one pass of the whole method on one synthetic system, inputs
already in HBM: draw the Gaussian multiplier G, form M = A G, block Gaussian
elimination (panels of 256), the two triangular solves, the back-transformation
x = G y, and FP64 iterative refinement until the normwise backward error
eta <= 1e-14 (at most 16 steps).  Paths: factors in FP64 or in FP32 on the
matrix cores (refinement always FP64), each with no pivoting (GENP, "f64",
"f32") or with partial pivoting confined to the diagonal blocks of at most 128
("f64p", "f32p"), refined classically or, for FP32 factors, by GMRES preconditioned
with the factors ("f32g", "f32pg"), and "f32xg": as "f32pg" with the product
M = A G on the BF16 matrix cores (G rounded to BF16, A split into two BF16
terms, FP32 accumulation).  The headline is the fastest path that reaches
eta <= 1e-14;
its speed-up over FP64 GENP is reported beside it.

Rate convention: (2/3 n^3 + 2 n^2 nrhs) flops per step (the standard count for
an LU solve), divided by the wall time of the whole step; the executed flops
(which add 2 n^3 - n^2 for M = A G) are reported beside it.

Workload: n = 16384, A = Q1 diag(sigma) Q2^T with Haar Q1, Q2 and
sigma_i = kappa^(-i/(n-1)), kappa = 10^(1 + 7u) drawn from the seed, one
N(0, 1) right-hand side.

Usage: python bench.py [--steps K] [--warmup W] [--n N] [--seed S]
       python bench.py --workload differentiation   (forward + backward through the
       solve: n = 8192, Toeplitz multiplier, 16 right-hand sides; one JSON line of its own)
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

METRIC = "factor+solve TFLOP/s n=16384: FP64 vs FP32 MFMA+IR at equal bwd error"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}  # MI355X dense MFMA TFLOP/s
ETA_TARGET = 1e-14

# HBM bytes of one product launch at n = 16384, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# passes scaled by a plain-copy calibration (FETCH x 2.000, WRITE x 1.000);
# profiles/k_gemm_fast_product_n16384_hbm_traffic.txt.  Valid only for the kernel source
# those counters were taken on (product_fingerprint).
TRAFFIC = {"n": 16384, "source": "k_gemm_fast + tile_coords (csrc/gemm.hip) + csrc/mfma.h",
           "sha256": "58b45b88b2ba4d113ec5a823e40f81d15f171ca135f8ccbf0c171f9a67185d88",
           "f64": {"fetch_kib": 351848686.4, "write_kib": 2099200.0},
           "f32": {"fetch_kib": 199430821.6, "write_kib": 1050836.8}}
# the same for the split-BF16 product (k_gemm_bf16x2, path f32xg)
TRAFFIC_BF16 = {"n": 16384, "source": "k_gemm_bf16x2 + tile_coords (csrc/gemm.hip)",
                "sha256": "84e34bad2ce2417152b2ab9234b22cb2ab011987019de5d783b4c87f9550ff8c",
                "fetch_kib": 45956590.5, "write_kib": 1061462.2}


def log(msg):
    sys.stderr.write("[bench %s] %s\n" % (time.strftime("%H:%M:%S"), msg))
    sys.stderr.flush()


def lu_solve_flops(n, nrhs):
    return 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nrhs


# name: (factor precision, row exchanges, refinement)
PATHS = {"f64": ("F64", "PIVOT_NONE", "ir"), "f32": ("F32", "PIVOT_NONE", "ir"),
         "f64p": ("F64", "PIVOT_BLOCK", "ir"), "f32p": ("F32", "PIVOT_BLOCK", "ir"),
         "f32g": ("F32", "PIVOT_NONE", "gmres"), "f32pg": ("F32", "PIVOT_BLOCK", "gmres"),
         "f32xg": ("F32_BF16X2", "PIVOT_BLOCK", "gmres")}


def run_path(rmge, torch, A, b, name, seed, steps, warmup, block, max_refine, max_iters):
    prec, pivot = (getattr(rmge, x) for x in PATHS[name][:2])
    method = PATHS[name][2]
    f = rmge.factor(A, kind=rmge.GAUSSIAN, seed=seed, block=block, prec=prec, pivot=pivot)

    def solve():
        if method == "gmres":
            return f.solve_gmres(b, max_iters=max_iters, restart=32, tol=ETA_TARGET, out=X)
        return f.solve(b, max_refine=max_refine, tol=ETA_TARGET, out=X)

    if not f.ok:
        raise RuntimeError("factorization broke down: status %d" % f.status)
    X = torch.empty_like(b)
    for i in range(warmup):
        f.refactor(A, seed)
        _, st = solve()
        log("%s warmup %d: eta %.2e after %d refinement steps" % (name, i, st["eta"], st["iters"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts, tms = [], []
    for i in range(steps):
        f.refactor(A, seed)
        tms.append(f.times())  # HIP-event phase times, read on the host (no device work)
        _, st = solve()
        sts.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = sts[-1]
    avg = {k: sum(t[k] for t in tms) / steps for k in tms[0]}
    log("%s: %.1f ms/step (draw %.2f, product %.2f, elimination %.2f ms), eta0 %.2e, eta %.2e, "
        "%d refinement steps" % (name, dt * 1e3, avg["ms_multiplier"], avg["ms_product"],
                                 avg["ms_factor"], st["eta0"], st["eta"], st["iters"]))
    fstats = f.stats()  # growth (a device pass), after the timed region
    f.close()
    return {
        "ms_per_step": dt * 1e3,
        "ms_draw": avg["ms_multiplier"],
        "ms_product": avg["ms_product"],
        "ms_elimination": avg["ms_factor"],
        "eta0": st["eta0"],
        "eta": st["eta"],
        "refine_steps": st["iters"],
        "converged": bool(st["eta"] <= ETA_TARGET),
        "growth": fstats["growth"],
    }


def _function_text(src, signature):
    """Source text of the function whose definition contains `signature`, from its
    template line through the closing brace at column 0."""
    i = src.index(signature)
    i = src.rfind("\ntemplate", 0, i) + 1
    return src[i:src.index("\n}\n", i) + 3]


def product_fingerprint():
    """sha256 over what the product kernel is compiled from: its own text, the tile
    mapping it calls and the matrix-core wrappers (dispatch code is not part of it)."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_1406_5802_amd", "csrc")
    with open(os.path.join(csrc, "gemm.hip")) as fh:
        gemm = fh.read()
    with open(os.path.join(csrc, "mfma.h")) as fh:
        mfma = fh.read()
    i = gemm.index("__device__ inline void tile_coords(")
    tiles = gemm[i:gemm.index("\n}\n", i) + 3]
    text = _function_text(gemm, "void k_gemm_fast(") + tiles + mfma
    return hashlib.sha256(text.encode()).hexdigest()


def bf16_fingerprint():
    """sha256 over what the split-BF16 product kernel is compiled from: its own text
    and the tile mapping it calls."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_1406_5802_amd", "csrc")
    with open(os.path.join(csrc, "gemm.hip")) as fh:
        gemm = fh.read()
    i = gemm.index("__device__ inline void tile_coords(")
    tiles = gemm[i:gemm.index("\n}\n", i) + 3]
    text = _function_text(gemm, "void k_gemm_bf16x2(") + tiles
    return hashlib.sha256(text.encode()).hexdigest()


def product_traffic(n, prec):
    """Counter-measured HBM bytes per product launch ("f64", "f32" or "bf16"), or None if
    they do not apply (another size, or the kernel changed since the counters were taken)."""
    if prec == "bf16":
        if n != TRAFFIC_BF16["n"] or bf16_fingerprint() != TRAFFIC_BF16["sha256"]:
            return None
        return (TRAFFIC_BF16["fetch_kib"] + TRAFFIC_BF16["write_kib"]) * 1024.0
    if n != TRAFFIC["n"] or product_fingerprint() != TRAFFIC["sha256"]:
        return None
    t = TRAFFIC[prec]
    return (t["fetch_kib"] + t["write_kib"]) * 1024.0


def cpu_baseline(n_cpu, seed, local_pivot_block=0):
    import numpy as np

    import oracle
    import workloads

    kappa = workloads.precision_kappa(seed)
    log("cpu baseline: generating the n=%d sample (same recipe, on the GPU)" % n_cpu)
    A = workloads.conditioned_torch(n_cpu, kappa, seed).cpu().numpy()
    b = workloads.rhs_torch(n_cpu, 1, seed).cpu().numpy()
    oracle.lib()
    log("cpu baseline: oracle factor + solve on %d threads" % oracle.num_threads())
    t0 = time.perf_counter()
    f = oracle.factor(A, oracle.GAUSSIAN, seed, local_pivot_block=local_pivot_block)
    s = oracle.solve(f, b, refine=1)
    dt = time.perf_counter() - t0
    log("cpu baseline: %.1f s, eta %.2e" % (dt, s.eta[-1]))
    return {
        "value": lu_solve_flops(n_cpu, 1) / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "n=%d system of the same recipe (Gaussian multiplier, %s, FP64, 1 RHS, 1 "
                  "refinement step), plain-loop C oracle; %.1f s wall"
                  % (n_cpu, "pivoting inside blocks of %d" % local_pivot_block
                     if local_pivot_block else "no pivoting", dt),
        "eta": float(s.eta[-1]),
        "seconds": dt,
    }


DIFF_PATHS = {"f64": ("F64", "PIVOT_NONE"), "f32p": ("F32", "PIVOT_BLOCK")}


def differentiation(args):
    """The differentiation workload: n = 8192, Toeplitz multiplier, 16 right-hand
    sides, loss sum(W .* X).  One step is the forward solve X = A^{-1} B (factor
    with the multiplier, solve, refine to eta <= 1e-14) and the backward pass
    (grad_B = A^{-T} W by the refined adjoint solve reusing the factors, then
    grad_A = -grad_B X^T), as torch.autograd runs them.  The roofline line is the
    grad_A kernel (HBM: writes n^2 doubles, reads 2 n nrhs)."""
    import torch

    import paper_1406_5802_amd as rmge
    from paper_1406_5802_amd import autograd
    import workloads

    rmge.lib()
    n, nrhs, kappa = args.n or 8192, 16, 1e2
    log("differentiation: n=%d Toeplitz multiplier, %d RHS, kappa=%g" % (n, nrhs, kappa))
    A = workloads.conditioned_torch(n, kappa, seed=args.seed)
    B = workloads.rhs_torch(n, nrhs, seed=args.seed)
    W = workloads.rhs_torch(n, nrhs, seed=args.seed + 1)
    torch.cuda.synchronize()
    paths = {}
    for name in args.paths.split(","):
        if name not in DIFF_PATHS:
            raise SystemExit("unknown differentiation path %r (choose from %s)"
                             % (name, ",".join(DIFF_PATHS)))
        prec, pivot = (getattr(rmge, x) for x in DIFF_PATHS[name])
        kw = dict(kind=rmge.TOEPLITZ, seed=args.seed + 1000, block=args.block, prec=prec,
                  pivot=pivot, tol=ETA_TARGET)
        fwd, bwd = [], []
        for i in range(args.warmup + args.steps):
            At = A.clone().requires_grad_(True)
            Bt = B.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X = autograd.solve(At, Bt, **kw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            (W * X).sum().backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if i >= args.warmup:
                fwd.append((t1 - t0) * 1e3)
                bwd.append((t2 - t1) * 1e3)
        paths[name] = {"ms_forward": sum(fwd) / len(fwd), "ms_backward": sum(bwd) / len(bwd)}
        paths[name]["ms_per_step"] = paths[name]["ms_forward"] + paths[name]["ms_backward"]
        log("%s: forward %.2f ms, backward %.2f ms" % (name, paths[name]["ms_forward"],
                                                       paths[name]["ms_backward"]))
        GB, Xd = Bt.grad.detach(), X.detach()
    # the grad_A kernel alone, on the stream the library is given (events around
    # each launch: the call synchronises that stream before it returns)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rmge.grad_A(GB, Xd)
    reps, ms_ga = 10, 0.0
    for _ in range(reps):
        e0.record()
        rmge.grad_A(GB, Xd)
        e1.record()
        e1.synchronize()
        ms_ga += e0.elapsed_time(e1) / reps
    ga_bytes = 8.0 * n * n + 2 * 8.0 * n * nrhs
    head = min(paths, key=lambda k: paths[k]["ms_per_step"])
    out = {
        "metric": "differentiation: forward+backward time, n=%d Toeplitz, %d RHS" % (n, nrhs),
        "value": round(paths[head]["ms_per_step"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(paths[head]["ms_per_step"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factors + f64 refinement" if head.startswith("f32") else "f64",
        "data": "synthetic",
        "config": {"workload": "differentiation: n=%d Toeplitz multiplier, %d RHS, kappa=%g, "
                               "loss sum(W .* X), eta<=1e-14" % (n, nrhs, kappa),
                   "n": n, "nrhs": nrhs, "kappa": kappa, "seed": args.seed, "block": args.block,
                   "headline_path": head},
        "roofline": {"bound": "hbm", "achieved": round(ga_bytes / (ms_ga * 1e-3) / 1e9, 1),
                     "peak": 8000.0, "unit": "GB/s",
                     "frac": round(ga_bytes / (ms_ga * 1e-3) / 1e9 / 8000.0, 4),
                     "traffic": None, "kernel": "k_grad_a (grad_A = -grad_B X^T)",
                     "ms_per_launch": round(ms_ga, 4)},
        "paths": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in paths.items()},
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision", choices=["precision", "differentiation"],
                    help="precision: the factor+solve benchmark (default); differentiation: "
                         "forward and backward through the solve at n = 8192, Toeplitz, 16 RHS")
    ap.add_argument("--n", type=int, default=None, help="16384 (precision) or 8192 "
                                                         "(differentiation)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--max-refine", type=int, default=16)
    ap.add_argument("--paths", default=None,
                    help="precision: f64,f32,f64p,f32p,f32g,f32pg,f32xg (default f64,f32,f64p,"
                         "f32p,f32pg,f32xg); differentiation: f64,f32p (default both)")
    ap.add_argument("--max-iters", type=int, default=200, help="GMRES inner iterations in all")
    ap.add_argument("--cpu-n", type=int, default=8192,
                    help="size of the oracle's CPU sample (about 20 s on 16 host threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--matrix", default="conditioned", choices=["conditioned", "gaussian"],
                    help="conditioned: Q1 diag(sigma) Q2^T (the workload); gaussian: i.i.d. "
                         "N(0, 1/n) entries, no QR (for hardware-counter passes, where only "
                         "the shape matters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the method is benchmarked on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "differentiation":
        args.paths = args.paths or "f64,f32p"
        return differentiation(args)
    args.paths = args.paths or "f64,f32,f64p,f32p,f32pg,f32xg"

    import torch

    import paper_1406_5802_amd as rmge
    import workloads

    rmge.lib()
    n = args.n or 16384
    kappa = workloads.precision_kappa(args.seed)
    if args.matrix == "gaussian":
        log("generating A: n=%d i.i.d. Gaussian (seed %d) on the GPU" % (n, args.seed))
        A = workloads.gaussian_torch(n, args.seed)
        kappa = None
    else:
        log("generating A: n=%d kappa=%.3g (seed %d) on the GPU" % (n, kappa, args.seed))
        A = workloads.conditioned_torch(n, kappa, args.seed)
    b = workloads.rhs_torch(n, 1, args.seed)
    torch.cuda.synchronize()
    log("inputs ready")

    results = {}
    for p in args.paths.split(","):
        if p not in PATHS:
            ap.error("unknown path %r (choose from %s)" % (p, ",".join(PATHS)))
        results[p] = run_path(rmge, torch, A, b, p, args.seed + 1000, args.steps, args.warmup,
                              args.block, args.max_refine, args.max_iters)

    ok = {k: v for k, v in results.items() if v["converged"]}
    head = min(ok, key=lambda k: ok[k]["ms_per_step"]) if ok else next(iter(results))
    r = results[head]
    fp32 = head.startswith("f32")
    split = PATHS[head][0] == "F32_BF16X2"
    flops = lu_solve_flops(n, 1)
    value = flops / (r["ms_per_step"] * 1e-3) / 1e12
    # roofline of the dominant kernel: the M = A G product, one launch per step.
    # Algorithmic flops 2 n^3 - n^2 in every case; the split-BF16 product executes
    # two BF16 products and is priced against the dense BF16 peak.
    prod_flops = 2.0 * n ** 3 - n * n
    achieved = prod_flops / (r["ms_product"] * 1e-3) / 1e12
    peak_key = "bf16" if split else ("f32" if fp32 else "f64")
    if split:
        kernel = "k_gemm_bf16x2 (M = A_h G + A_l G, BF16 MFMA, FP32 accumulation)"
        traffic = product_traffic(n, "bf16")
    else:
        kernel = "k_gemm_fast<%s, 2, 0> (M = A G)" % ("float, float" if fp32 else "double, double")
        traffic = product_traffic(n, "f32" if fp32 else "f64")
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("bf16x2 product + f32 factors (bf16x3 Schur updates) + f64 refinement" if split else
                  "f32 factors + f64 refinement" if fp32 else "f64"),
        "data": "synthetic",
        "config": {"workload": ("precision: n=%d Gaussian multiplier, kappa=%.3g, 1 RHS, "
                                "eta<=1e-14" % (n, kappa)) if kappa else
                               ("n=%d i.i.d. Gaussian A, Gaussian multiplier, 1 RHS, "
                                "eta<=1e-14" % n),
                   "n": n, "kappa": kappa, "seed": args.seed, "block": args.block, "nrhs": 1,
                   "headline_path": head},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK[peak_key], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK[peak_key], 4),
                     "traffic": traffic,
                     "traffic_unit": "bytes/launch",
                     "kernel": kernel,
                     "ms_per_launch": round(r["ms_product"], 4)},
        "executed_tflops": round((flops + prod_flops) / (r["ms_per_step"] * 1e-3) / 1e12, 3),
        "paths": {k: {kk: (float("%.6g" % vv) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in results.items()},
    }
    if "f64" in results and head != "f64":
        out["speedup_over_f64_genp"] = round(results["f64"]["ms_per_step"] / r["ms_per_step"], 3)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.seed,
                                           args.block if head.endswith("p") else 0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
