#!/usr/bin/env python3
"""SpAMM on one MI355X: time and leaf TFLOP/s at relative error 1e-6, vs dense GEMM.

Workload: algebraic decay a_ij = u_ij / (|i-j|^2 + 1), u ~ U(0.5, 1.5)
(seeded counter-based draws), n = 8192, leaf 64, FP32 storage, C = A A.
For every leaf precision the largest tau on a quarter-decade grid whose
product meets ||C~ - C||_F / ||C||_F <= 1e-6 is found against the exact
product (FP64 leaves at tau = 0, on the GPU); the fastest precision that
meets the target is timed.

A timed step is one pass of the hot path over resident inputs: quadtree
build of A (pack + FP64 norm pyramid) and the SpAMM product (cull, leaf
products, result norm pyramid).  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpAMM time & leaf TFLOP/s at rel. err 1e-6 vs dense GEMM, 1 MI355X"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "bf16x3": 2516.6, "f16": 2516.6, "f16x3": 2516.6}
HW_MULT = {"f64": 1, "f32": 1, "bf16": 1, "bf16x3": 3, "f16": 1, "f16x3": 3}


# HBM bytes per leaf launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs
# (KiB per dispatch, n = 8192, leaf 64, tau = 1e-6), scaled by the factors a
# 256 MiB device copy gives in the same runs (FETCH x 2.0, WRITE x 1.0).  The
# figures belong to one version of the leaf kernel source: when the source
# hash differs they are not reported.
PMC_TRAFFIC = {
    "src_sha256_16": "11434a1fe4cd4d32",
    "fetch_factor": 2.0, "write_factor": 1.0,
    "leaf": {("f16x3", 64, 8192, 1e-6): (860988.0, 262805.5), ("f32", 64, 8192, 1e-6): (858665.1, 262810.7)},
}


def leaf_traffic(prec, leaf, n, tau):
    import hashlib
    src = os.path.join(ROOT, "paper_1011_3534_amd", "csrc", "leaf.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    key = (prec, leaf, n, float(f"{tau:.3g}"))
    if sha != PMC_TRAFFIC["src_sha256_16"] or key not in PMC_TRAFFIC["leaf"]:
        return None
    f, w = PMC_TRAFFIC["leaf"][key]
    return (f * PMC_TRAFFIC["fetch_factor"] + w * PMC_TRAFFIC["write_factor"]) * 1024.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tau_grid(hi=1e-4, lo=1e-9):
    k = 0
    out = []
    while True:
        t = hi * 10 ** (-k / 4)
        if t < lo * 0.999:
            return out
        out.append(float(f"{t:.3g}"))
        k += 1


def cpu_baseline(a64, leaf, tau, seconds):
    """The FP64 oracle's flat SpAMM timed on a bounded sample of C tile rows."""
    import oracle
    nb = a64.shape[0] // leaf

    def timed(rows):
        t0 = time.perf_counter()
        oracle.spamm_flat(a64, a64, leaf, tau, rows=(nb // 2, nb // 2 + rows))
        return time.perf_counter() - t0

    t1, t3 = timed(1), timed(3)
    per_row = max((t3 - t1) / 2, 1e-3)
    fixed = max(t1 - per_row, 0.0)
    rows = int(max(1, min(nb, (seconds - fixed) / per_row)))
    r0 = max(0, nb // 2 - rows // 2)
    t0 = time.perf_counter()
    _, T = oracle.spamm_flat(a64, a64, leaf, tau, rows=(r0, r0 + rows))
    dt = time.perf_counter() - t0
    flops = 2.0 * leaf ** 3 * T
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"C tile rows [{r0},{r0 + rows}) of {nb} ({T} leaf products, {dt:.1f} s, FP64, "
                      f"norms of the whole operand included)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--target", type=float, default=1e-6)
    ap.add_argument("--precisions", default="f32,f16x3,bf16x3,f16,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--tau", type=float, default=None,
                    help="use this tau for every precision instead of the sweep (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has no "
              f"multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1011_3534_amd as sp
    import spamm_inputs as si

    torch.cuda.set_device(0)
    sp.use_torch_allocator(True)
    n, b = args.n, args.leaf
    log(f"generating n={n} algebraic-decay operand")
    a = si.algebraic_workload(n)
    A_d = torch.from_numpy(a).cuda()
    A = sp.build(A_d, b)
    log("exact product (FP64 leaves, tau = 0)")
    E = sp.multiply(A, A, 0.0, "f64")
    torch.cuda.synchronize()

    # dense FP32 GEMM comparator (torch -> hipBLASLt/rocBLAS)
    for _ in range(3):
        Cd = torch.matmul(A_d, A_d)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    ev0.record()
    for _ in range(reps):
        Cd = torch.matmul(A_d, A_d)
    ev1.record()
    torch.cuda.synchronize()
    dense_ms = ev0.elapsed_time(ev1) / reps
    Dh = sp.build(Cd, b)
    dense_err = sp.rel_err(Dh, E)
    Dh.free()
    log(f"dense FP32 GEMM {dense_ms:.3f} ms, rel err {dense_err:.2e}")

    # tau per precision
    precs = {}
    grid = tau_grid() if args.tau is None else [args.tau]
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    for p in args.precisions.split(","):
        C = None
        found = None
        sweep = []
        for tau in grid:
            C, st = sp.multiply(A, A, tau, p, out=C, stats=True)
            err = sp.rel_err(C, E)
            sweep.append((tau, err, st["tasks"]))
            if err <= args.target or args.tau is not None:
                found = (tau, err, st["tasks"])
                break
        precs[p] = {"handle": C, "found": found, "sweep": sweep}
        log(f"{p}: " + (f"tau*={found[0]:.3g} err={found[1]:.2e} T={found[2]}" if found
                         else f"misses {args.target:g} (floor {sweep[-1][1]:.2e})"))

    # time each qualifying precision: whole step, and the leaf launch alone
    results = {}
    for p, d in precs.items():
        if d["found"] is None:
            continue
        tau, err, T = d["found"]
        C = d["handle"]
        for _ in range(args.warmup):
            sp.build(A_d, b, out=A)
            sp.multiply(A, A, tau, p, out=C)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            sp.build(A_d, b, out=A)
            sp.multiply(A, A, tau, p, out=C)
        ev1.record()
        torch.cuda.synchronize()
        step_ms = ev0.elapsed_time(ev1) / args.steps
        phases = [sp.multiply_timed(A, A, tau, p, out=C)[1] for _ in range(args.steps)]
        leaf_ms = float(np.mean([ph["ms_leaf"] for ph in phases]))
        cull_ms = float(np.mean([ph["ms_cull"] for ph in phases]))
        mult_ms = float(np.mean([ph["ms_total"] for ph in phases]))
        flops = 2.0 * b ** 3 * T
        results[p] = {"tau": tau, "rel_err": err, "tasks": T, "step_ms": step_ms, "multiply_ms": mult_ms,
                      "leaf_ms": leaf_ms, "cull_ms": cull_ms, "leaf_tflops": flops / leaf_ms / 1e9,
                      "step_tflops": flops / step_ms / 1e9, "speedup_vs_dense_fp32": dense_ms / step_ms}
        log(f"{p}: step {step_ms:.3f} ms (multiply {mult_ms:.3f}, leaf {leaf_ms:.3f}, cull {cull_ms:.3f}) "
            f"leaf {flops / leaf_ms / 1e9:.1f} TFLOP/s")

    if not results:
        print(json.dumps({"metric": METRIC, "value": None, "error": "no precision met the target"}))
        sys.exit(1)
    best = min(results, key=lambda p: results[p]["step_ms"])
    r = results[best]
    achieved = r["leaf_tflops"]
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[best], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[best], 4), "traffic": leaf_traffic(best, b, n, r["tau"]),
            "kernel": f"k_leaf<{b},{best}>", "hw_flop_mult": HW_MULT[best],
            "hw_frac": round(achieved * HW_MULT[best] / PEAK_TFLOPS[best], 4)}
    out = {"metric": METRIC, "value": round(r["step_tflops"], 3), "unit": "TFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["step_ms"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": best,
           "data": "synthetic",
           "config": {"workload": f"algebraic decay u/(|i-j|^2+1), u~U(0.5,1.5), n={n}, leaf {b}, FP32 storage, "
                                  f"C=A*A, tau for rel. err <= {args.target:g}",
                      "n": n, "leaf": b, "tau": r["tau"], "leaf_precision": best},
           "rel_err": r["rel_err"], "tasks": r["tasks"], "leaf_tflops": round(achieved, 3),
           "spamm_step_ms": round(r["step_ms"], 4), "dense_fp32_gemm_ms": round(dense_ms, 4),
           "dense_fp32_rel_err": dense_err, "speedup_vs_dense_fp32": round(dense_ms / r["step_ms"], 3),
           "precisions": {p: {k: (float(f"{v:.5g}") if isinstance(v, float) else v) for k, v in res.items()}
                          for p, res in results.items()},
           "missed_target": {p: {"floor_rel_err": d["sweep"][-1][1]} for p, d in precs.items()
                             if d["found"] is None},
           "roofline": roof}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(a.astype(np.float64), b, r["tau"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
