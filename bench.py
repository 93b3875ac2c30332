#!/usr/bin/env python3
"""Benchmark of the Mat2Stencil hot path on one MI355X.

Workload (default): the 256^3 HPCG-style 27-point operator with a 4-level
multigrid V-cycle (1 pre- and 1 post-SymGS per level, injection transfers)
preconditioning CG; b = A*1 + N(0, 1e-3) (seed 3), x0 = 0.  Synthetic
stand-in for HPCG; no dataset involved.

A "step" is one MG-PCG iteration (V-cycle: 8 level-0 half-sweeps' worth of
SymGS plus SpMV, restriction, prolongation on every level; top-level SpMV,
three dot products and three vector updates).  `value` is GFLOP/s in the
HPCG convention (2 flops per stored non-zero per SpMV or sweep direction,
2 per vector element per dot/axpy) over the timed steps.

Also reported on the same line:
  roofline      the exact lexicographic SymGS wavefront kernel at 256^3
                (forward half-sweep out of place: algorithmic 24 B/point),
                timed with HIP events on its stream, against 8 TB/s;
  spmv          the 27-point SpMV kernel (16 B/point) likewise;
  time_to_solution  FP64 MG-PCG and mixed-precision MG-PCG (FP32 V-cycle,
                FP64 CG) to relative residual 1e-9 from x0 = 0;
  cpu_baseline  the CPU oracle (single thread) on a bounded sample.

    python bench.py [--gpus 1] [--steps 50] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU-oracle baseline")
    ap.add_argument("--no-tts", action="store_true",
                    help="skip the time-to-solution runs")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the kernel roofline loops (for profiling)")
    return ap.parse_args()


def nnz27(n):
    return (3 * n - 2) ** 3


def flops_per_iteration(n, levels):
    """HPCG convention for one MG-PCG iteration on an n^3 grid."""
    f = 0
    for lv in range(levels):
        m = n >> lv
        if lv < levels - 1:
            f += (4 + 2 + 4) * nnz27(m)  # pre SymGS, residual, post SymGS
        else:
            f += 4 * nnz27(m)            # coarsest SymGS
    f += 2 * nnz27(n)                    # Ap
    f += 3 * 2 * n ** 3                  # three dot products
    f += 3 * 2 * n ** 3                  # x, r, p updates
    return f


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def event_time_ms(torch, fn, reps):
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
        enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                          "--gpus must be 1 (multi-GPU sharding is "
                          "described in DESIGN.md, not implemented)"}))
        return 2
    import numpy as np
    import torch

    import paper_2204_13304_amd as m
    from paper_2204_13304_amd import inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    dev = torch.device("cuda:0")
    n, L = args.n, args.levels
    shape = (n, n, n)
    npts = n ** 3
    log(f"setup {shape} levels={L}")
    A = m.const27(shape)
    ones = torch.ones(shape, dtype=torch.float64, device=dev)
    b = m.spmv(A, ones)
    b += torch.from_numpy(inputs.rhs_perturbation(3, shape)).to(dev)
    torch.cuda.synchronize()

    # ---------------------------------------------------------- roofline
    ws = m.Workspace(A)
    r = torch.from_numpy(inputs.standard_normal(10, shape)).to(dev)
    x0 = torch.from_numpy(inputs.standard_normal(11, shape)).to(dev)
    x1 = torch.empty_like(x0)
    for _ in range(3):
        m.symgs_oop(A, r, x0, x1, "fwd", ws)
    reps = 20
    sweep_ms = event_time_ms(torch, lambda: m.symgs_oop(A, r, x0, x1, "fwd",
                                                         ws), reps)
    ws.check()
    sweep_bytes = 24 * npts
    sweep_gbs = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    spmv_ms = event_time_ms(torch, lambda: m.spmv(A, x0, x1), reps)
    spmv_gbs = 16 * npts / (spmv_ms * 1e-3) / 1e9
    log(f"sweep {sweep_ms:.3f} ms {sweep_gbs:.0f} GB/s; spmv {spmv_ms:.3f} ms "
        f"{spmv_gbs:.0f} GB/s")
    if args.roofline_only:
        print(json.dumps({"sweep_ms": sweep_ms, "spmv_ms": spmv_ms}))
        return 0

    # ---------------------------------------------------------- steps
    mg = m.MG(A, L)
    x = torch.zeros_like(b)
    log(f"warmup {args.warmup}")
    if args.warmup > 0:
        m.pcg_solve(A, b, x, "mg", mg, max_iter=args.warmup, rtol=0.0)
    x.zero_()
    torch.cuda.synchronize()
    log(f"timed {args.steps} MG-PCG iterations")
    t0 = time.perf_counter()
    _, info = m.pcg_solve(A, b, x, "mg", mg, max_iter=args.steps, rtol=0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gflops = flops_per_iteration(n, L) * args.steps / (t1 - t0) / 1e9
    log(f"{ms_per_step:.3f} ms/iteration, {gflops:.1f} GFLOP/s, "
        f"relres {info['rel_res']:.3e}")

    # ---------------------------------------------------------- TTS
    tts = None
    if not args.no_tts:
        out = {}
        for tag, prec, rep in (("fp64", torch.float64, 0),
                               ("mixed", torch.float32, 50)):
            mgp = m.MG(A, L, prec=prec)
            xs = torch.zeros_like(b)
            m.pcg_solve(A, b, xs, "mg", mgp, max_iter=2, rtol=0.0)  # warm
            xs.zero_()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, inf = m.pcg_solve(A, b, xs, "mg", mgp, max_iter=500,
                                 rtol=1e-9, replace_every=rep)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            out[tag] = dict(seconds=tb - ta, iters=inf["iters"],
                            true_rel_res=inf["true_rel_res"])
            out[tag + "_x"] = xs
            log(f"tts {tag}: {tb - ta:.4f} s, {inf['iters']} it, "
                f"true relres {inf['true_rel_res']:.2e}")
        err = (out["mixed_x"] - out["fp64_x"]).abs().max().item() / \
            out["fp64_x"].abs().max().item()
        tts = dict(rtol=1e-9, fp64=out["fp64"], mixed=out["mixed"],
                   speedup_mixed=out["fp64"]["seconds"] /
                   out["mixed"]["seconds"],
                   mixed_vs_fp64_rel_err=err)

    # ---------------------------------------------------------- CPU
    cpu = None
    if not args.no_cpu:
        try:
            import oracle
            bh = b.cpu().numpy()
            log("cpu oracle: 1 and 2 MG-PCG iterations")
            ta = time.perf_counter()
            oracle.pcg(bh, precond="mg", levels=L, max_iter=1)
            tb = time.perf_counter()
            oracle.pcg(bh, precond="mg", levels=L, max_iter=2)
            tc = time.perf_counter()
            per_it = max(1e-9, (tc - tb) - (tb - ta))
            cpu = {"value": flops_per_iteration(n, L) / per_it / 1e9,
                   "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                   "sample": f"one MG-PCG iteration at {n}^3 (difference "
                             "of a 2-iteration and a 1-iteration oracle "
                             f"run; {per_it:.2f} s per iteration)"}
        except Exception as e:  # report, do not hide
            cpu = {"error": repr(e)}

    line = {
        "metric": "SymGS+SpMV GFLOP/s (HPCG convention) in 256^3 MG-PCG; "
                  "% HBM roofline of the SymGS sweep; MG-PCG time-to-1e-9 "
                  "FP64 vs mixed",
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"const27 {n}^3 {L}-level MG-PCG, b = A*1 + "
                               "N(0,1e-3) seed 3, x0 = 0",
                   "grid": [n, n, n], "levels": L},
        "roofline": {"bound": "hbm", "achieved": sweep_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sweep_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_wave_kernel<CONST27,double,fwd> "
                               f"{n}^3, 24 B/point",
                     "avg_ms": sweep_ms},
        "spmv": {"achieved": spmv_gbs, "unit": "GB/s", "avg_ms": spmv_ms,
                 "frac": spmv_gbs / HBM_PEAK_GBS},
        "time_to_solution": tts,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
