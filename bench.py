"""Benchmark: V-cycle-preconditioned CG on the 3-D ball, one MI355X.

One step = one CG solve to ||r|| <= 1e-8 ||b|| with the multigrid V-cycle
(coloured multiplicative vertex-patch smoother, matrix-free Nitsche + ghost
penalty operator, transfers, exact coarse solve) on the ball |x| < 0.7 cut from
[-1, 1]^3, Q2, 6 levels up to 128^3 cells (3,246,717 active DoFs), FP64.
Inputs are synthetic (manufactured right-hand side) and resident in HBM before
the timed region starts.

value = V-cycle DoFs/s = active DoFs x V-cycles applied / wall time of the timed
solves (the CG work around the V-cycles is included).

roofline: the dominant kernel (default: the cut-patch colour step) is bracketed
by HIP events on its own stream during the timed region; achieved = algorithmic
bytes of its launches / their summed duration, against 8 TB/s.

cpu_baseline: the CPU oracle (NumPy/SciPy, one thread) solving the same problem
on a bounded sample: the same ball at 32^3 cells (4 levels, 62,801 DoFs).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "V-cycle DoFs/s FP64 vs FP32-precond at 1e-8 rel residual; p50/p99 solve latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ball", choices=["ball", "disc"])
    ap.add_argument("--levels", type=int, default=None, help="override the level count (smaller runs)")
    ap.add_argument("--kernel", default="cut_solve", choices=["cut_solve", "interior_step", "apply"],
                    help="kernel kind whose roofline is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--fp32", action="store_true", help="FP32 multigrid preconditioner inside FP64 CG")
    return ap.parse_args()


def kernel_source_hash() -> str:
    src = os.path.join(ROOT, "paper_2508_11608_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def algorithmic_bytes(P, w, kind: str) -> dict:
    """Algorithmic HBM bytes of every launch of one kernel kind in one V-cycle,
    keyed by (level, colour) (or level for 'apply'), FP64 (s = 8 B).

    interior_step, per patch:  s [(2k)^d + 2 (2k-1)^d] + 4
        x over the patch closure (same-coloured closures tile space with period
        2k nodes), b on the internal nodes, x written on them, vertex index.
    cut_solve, per patch j:    s N_j^2 + N_j (4 + 2 s) + 12 + s (2k)^d
                               + s k^d (k+1)^d x (cut cells of the patch)
        dense inverse, node list, b and correction, offsets, x over the
        closure, and the k^d rows of every cut-cell matrix that belong to
        internal nodes of the patch.
    apply (residual), per DoF: 4 + 3 s, plus s (k+1)^{2d} per cut cell; the
        CG product A p once per iteration on the finest level: 4 + 2 s per DoF.
    """
    s = 8
    d, k = w.dim, w.k
    nl = (k + 1) ** d
    out = {}
    for l in range(1, w.n_levels):
        c = P.counts(l)
        if kind == "apply":
            out[l] = c["n_dofs"] * (4 + 3 * s) + c["cut_cells"] * nl * nl * s
            if l == w.n_levels - 1:  # the CG product A p on the finest level (no b)
                out["cg"] = c["n_dofs"] * (4 + 2 * s) + c["cut_cells"] * nl * nl * s
            continue
        N = P.export(l, 2, np.uint8)  # cell flags, x fastest
        Nc = round(len(N) ** (1.0 / d))
        flags = N.reshape((Nc,) * d)  # index order (z, y, x) / (y, x)
        cut = (flags & 2) != 0
        for col in range(2 ** d):
            if kind == "interior_step":
                nv = len(P.export(l, 16 + col, np.int32))
                if nv:
                    out[(l, col)] = nv * (s * ((2 * k) ** d + 2 * (2 * k - 1) ** d) + 4)
                continue
            off = P.export(l, 24 + col, np.int32)
            verts = P.export(l, 48 + col, np.int32)
            if len(verts) == 0:
                continue
            nj = np.diff(off).astype(np.int64)
            NV = Nc + 1
            V = np.stack([(verts // NV ** i) % NV for i in range(d)], axis=1)  # (x, y[, z])
            ncut = np.zeros(len(verts), dtype=np.int64)
            for o in range(2 ** d):
                ci = V - 1 + np.array([(o >> i) & 1 for i in range(d)])
                ok = np.all((ci >= 0) & (ci < Nc), axis=1)
                idx = tuple(ci[ok][:, i] for i in reversed(range(d)))
                ncut[ok] += cut[idx]
            b = (s * nj ** 2 + nj * (4 + 2 * s) + 12 + s * (2 * k) ** d + s * k ** d * nl * ncut).sum()
            out[(l, col)] = int(b)
    return out


def roofline(P, w, kind: str, launches: int, total_ms: float, vcycles: int) -> dict:
    per_v = algorithmic_bytes(P, w, kind)
    bytes_per_vcycle = sum(per_v.values())
    if kind != "apply":
        # each colour step runs twice per smoothing step for interior patches
        # (pre + post) and 2 n_c times for cut patches
        bytes_per_vcycle *= 2 if kind == "interior_step" else 2 * w.n_c
    launches_per_v = launches / max(vcycles, 1)
    bytes_per_launch = bytes_per_vcycle / max(launches_per_v, 1e-30)
    ms_per_launch = total_ms / max(launches, 1)
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kind}_{w.name}.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("kernel_source_sha256_16") == kernel_source_hash():
            traffic = t.get("bytes_per_launch")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kind,
            "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_us": ms_per_launch * 1e3,
            "launches_timed": launches}


def cpu_baseline() -> dict:
    """The CPU oracle as it stands, one thread, on the 32^3 ball (4 levels)."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import problem as OP
    from oracle.multigrid import pcg

    w = W.ball_q2().with_levels(4)
    with threadpool_limits(limits=1):
        levels, mats, _, H = OP.build(w)
        b = OP.rhs(w, levels[-1])
        n = levels[-1].n_dofs
        its = 0
        t0 = time.perf_counter()
        solves = 0
        while solves < 3 or time.perf_counter() - t0 < 10.0:  # at least 3 solves and 10 s
            _, it, _ = pcg(mats[-1], b, H.vcycle, rtol=1e-8)
            its += it
            solves += 1
        dt = time.perf_counter() - t0
    return {"value": n * its / dt, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"{solves} FP64 PCG solves to 1e-8 on the same ball at 32^3 cells (4 levels, {n} DoFs, "
                      f"{its // solves} iterations each), set-up excluded, {dt:.1f} s"}


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
    P = Problem(w, fp32=args.fp32)
    t_setup = time.perf_counter() - t0
    n = P.ndofs()
    print(f"[bench] {w.name}: {n} DoFs, setup {t_setup:.1f}s", file=sys.stderr, flush=True)
    b = torch.from_numpy(P.rhs_manufactured()).cuda()
    x = torch.empty_like(b)
    for _ in range(args.warmup):
        P.solve(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    P.timing([args.kernel])
    its = 0
    rel = None
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, info = P.solve(b, x, rtol=1e-8)
        lat.append(time.perf_counter() - ts)
        its += info["iterations"]
        rel = info["rel_residual"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms = P.timing_read(args.kernel)
    P.timing([])
    roof = roofline(P, w, args.kernel, launches, kms, its)
    print(f"[bench] timed {args.steps} solves: {dt:.3f}s, {its} V-cycles", file=sys.stderr, flush=True)
    # back-to-back V-cycles only (outside the timed region)
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
        "metric": METRIC,
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
        "config": {"workload": f"{w.name}: ball |x|<0.7 in [-1,1]^3, Q2, {w.n_levels} levels to "
                               f"{w.fine_cells}^3 cells, manufactured f, FP64 CG to 1e-8",
                   "active_dofs": n, "n_c": w.n_c, "precision": "fp64"},
        "roofline": roof,
        "cg_iterations_per_solve": its / args.steps,
        "final_rel_residual": rel,
        "solve_latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "solve_latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "vcycle_ms": t_v * 1e3,
        "vcycle_dofs_per_s": n / t_v,
        "setup_s": t_setup,
    }
    if args.fp32:
        out["dtype"] = "f32 multigrid in f64 CG"
        out["config"]["precision"] = "fp32 preconditioner, fp64 CG"
    P.close()
    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes_each_way"] = src.numel() * 8
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
