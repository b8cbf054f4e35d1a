"""Benchmark: V-cycle-preconditioned CG on the 3-D ball, one MI355X.

One step = one FP64 CG solve to ||r|| <= 1e-8 ||b|| with the multigrid V-cycle
(coloured multiplicative vertex-patch smoother, matrix-free Nitsche + ghost
penalty operator, transfers, exact coarse solve) on the ball |x| < 0.7 cut from
[-1, 1]^3, Q2, 6 levels up to 128^3 cells (3,246,717 active DoFs).  Inputs are
synthetic (manufactured right-hand side) and resident in HBM before timing.

value = V-cycle DoFs/s = active DoFs x V-cycles applied / time of the timed
solves (CG work included).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ball", choices=["ball", "disc"])
    ap.add_argument("--levels", type=int, default=None, help="override the level count (smaller runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU decomposition is a design note, "
              "not an implementation", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2508_11608_amd import Problem

    w = W.ball_q2() if args.workload == "ball" else W.disc_q2()
    if args.levels:
        w = w.with_levels(args.levels)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    P = Problem(w)
    t_setup = time.perf_counter() - t0
    n = P.ndofs()
    print(f"[bench] {w.name}: {n} DoFs, setup {t_setup:.1f}s", file=sys.stderr, flush=True)
    b = torch.from_numpy(P.rhs_manufactured()).cuda()
    x = torch.empty_like(b)
    for _ in range(args.warmup):
        P.solve(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    its = 0
    rel = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = P.solve(b, x, rtol=1e-8)
        its += info["iterations"]
        rel = info["rel_residual"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # back-to-back V-cycles only
    r = torch.randn(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    for _ in range(3):
        P.vcycle(r, z)
    torch.cuda.synchronize()
    nv = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(nv):
        P.vcycle(r, z)
    e1.record()
    torch.cuda.synchronize()
    t_v = e0.elapsed_time(e1) / 1e3 / nv
    out = {
        "metric": "V-cycle DoFs/s FP64 vs FP32-precond at 1e-8 rel residual; p50/p99 solve latency",
        "value": n * its / dt,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "k": w.k, "levels": w.n_levels,
                   "fine_cells": w.fine_cells, "active_dofs": n, "rtol": 1e-8, "n_c": w.n_c,
                   "precision": "fp64"},
        "cg_iterations_per_solve": its / args.steps,
        "final_rel_residual": rel,
        "vcycle_ms": t_v * 1e3,
        "vcycle_dofs_per_s": n / t_v,
        "setup_s": t_setup,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
