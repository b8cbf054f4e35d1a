"""Benchmark: V-cycle-preconditioned CG on the 3-D ball, one MI355X.

One step = one CG solve to ||r|| <= 1e-8 ||b|| with the multigrid V-cycle
(coloured multiplicative vertex-patch smoother, matrix-free Nitsche + ghost
penalty operator, transfers, exact coarse solve) on the ball |x| < 0.7 cut from
[-1, 1]^3, Q2, 6 levels up to 128^3 cells (3,246,717 active DoFs), FP64.
Inputs are synthetic (manufactured right-hand side) and resident in HBM before
the timed region starts.

value = V-cycle DoFs/s = active DoFs x V-cycles applied / wall time of the timed
solves (the CG work around the V-cycles is included).  Both precisions of the
multigrid are measured on the same hierarchy: the FP64 figures head the line
and the FP32-preconditioned ones (FP32 V-cycle inside FP64 CG, same 1e-8
tolerance) sit under "fp32_precond" (--fp32 swaps the two).

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
DOMAINS = {"ball": "ball |x|<0.7", "disc": "disc |x|<0.7",
           "union8": "union of 8 spheres (centres U[-0.6,0.6]^3, radii U[0.15,0.35], seed 0)"}
METRIC = "V-cycle DoFs/s FP64 vs FP32-precond at 1e-8 rel residual; p50/p99 solve latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ball", choices=["ball", "disc", "union8"],
                    help="ball: |x|<0.7, Q2, 128^3; disc: |x|<0.7, Q2, 32^2; union8: 8 seeded spheres, Q3, 64^3")
    ap.add_argument("--levels", type=int, default=None, help="override the level count (smaller runs)")
    ap.add_argument("--kernel", default="cut_solve", choices=["cut_solve", "interior_step", "apply"],
                    help="kernel kind whose roofline is reported")
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides per solve (up to 8): seeded Fourier loads, one multi-column PCG")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--fp32", action="store_true",
                    help="head the line with the FP32 multigrid preconditioner (FP64 figures go under 'fp64')")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="serving run: N seeded requests with Poisson arrivals instead of the solve benchmark")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--group", type=int, default=0, metavar="G",
                    help="grouped-V-cycle run: G problems of one lattice shape, alone against grouped")
    ap.add_argument("--ghost-sweep", default="", metavar="LEVELS",
                    help="the paper's ghost-parameter study (gamma_1 for Q1, then gamma_2 for Q2, then gamma_3 for Q3 "
                         "over 0.05..0.15) with fractional GMRES counts, for the comma-separated finest levels L")
    ap.add_argument("--paper-tables", default="", metavar="LEVELS",
                    help="iteration counts of GMRES and of the stand-alone V-cycle on the paper's circle protocol "
                         "for the comma-separated finest levels L (k = 1..3, n_c = 1..4), beside the paper's numbers")
    ap.add_argument("--rate", type=float, default=0.8, help="arrival rate as a fraction of the saturation rate")
    ap.add_argument("--small-cut-launch", type=int, default=None,
                    help="cut colour steps with fewer patches run with twice the threads per patch (default 1536)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every V-cycle kernel by kernel instead of replaying captured HIP graphs")
    return ap.parse_args()


def serve(args):
    """Continuous-batching run: the seeded request stream (unions of 1-4
    spheres or ellipsoids, d in {2,3}, k in {1,2,3}, N_L in {32,64,128}, random
    Fourier f, FP32 multigrid in FP64 CG to 1e-8) against one long-running
    server of the library.  Three phases on the same server: a cold pass (one
    request per distinct geometry: host set-up and admission), all requests at
    once (saturation throughput, the reported value), then the same stream with
    Poisson arrivals at `rate` x the saturation rate (the reported latencies)."""
    import workloads as W
    from paper_2508_11608_amd import Server

    reqs = W.serving_stream(args.serve, seed=0, pool=16, max_dofs=20_000_000)
    srv = Server(96 << 30, args.slots)

    def run(stream, arrivals, tag):
        t0 = time.perf_counter()
        pending = {}
        out = []
        i = 0
        while i < len(stream) or pending:
            now = time.perf_counter() - t0
            while i < len(stream) and arrivals[i] <= now:
                w, f = stream[i]
                pending[srv.submit(w, fourier=f, fp32=True)] = (i, w, time.perf_counter() - t0)
                i += 1
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    k, w, ts = pending.pop(t)
                    out.append((k, w, ts, time.perf_counter() - t0, r[0]))
                    print(f"[serve {tag}] {len(out)}/{len(stream)} request {k} {w.name}: status {r[0]['status']}, "
                          f"{r[0]['iterations']} its, batch {r[0]['batch']}, group {r[0]['group']}, "
                          f"{out[-1][3] - ts:.3f} s",
                          file=sys.stderr, flush=True)
            time.sleep(0.0005)
        return out, time.perf_counter() - t0

    first = {}
    for w, f in reqs:
        first.setdefault(w.name, (w, f))
    cold_out, cold_wall = run(list(first.values()), [0.0] * len(first), "cold")
    cold_lat = np.array([done - ts for _, _, ts, done, _ in cold_out])
    out, wall = run(reqs, [0.0] * len(reqs), "saturation")
    sat_rate = len(reqs) / wall
    dofs = sum(r["n_dofs"] * r["iterations"] for *_, r in out)
    sat_batch = [r["batch"] for *_, r in out]
    sat_group = sum(r["group"] > 1 for *_, r in out)
    rng = np.random.default_rng(1)
    arr = np.cumsum(rng.exponential(1.0 / (args.rate * sat_rate), len(reqs)))
    arr -= arr[0]
    out, p_wall = run(reqs, list(arr), "poisson")
    srv.close()
    lat = np.array([done - ts for _, _, ts, done, _ in out])
    solve = np.array([r["t_done"] - r["t_solve_start"] for *_, r in out])
    ok = all(r["status"] == 0 and r["rel_residual"] <= 1e-8 for *_, r in out)
    return {
        "metric": METRIC, "value": dofs / wall, "unit": "DoF/s (aggregate, per CG iteration)", "n_gpus": 1,
        "steps": len(reqs), "warmup": len(first), "ms_per_step": wall / len(reqs) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 multigrid in f64 CG", "data": "synthetic",
        "config": {"workload": f"serving stream: {len(reqs)} seeded requests, 16-geometry Zipf(1.1) pool "
                               f"({len(first)} distinct), unions of 1-4 spheres/ellipsoids, d in (2,3), k in (1,2,3), "
                               f"N_L in (32,64,128) (background lattice <= 2e7), Fourier f, rtol 1e-8, "
                               f"{args.slots} slots; value = saturation throughput on the warm server, latencies "
                               f"from Poisson arrivals at {args.rate} x saturation ({args.rate * sat_rate:.2f} req/s)"},
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3), "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "solve_ms_p50": float(np.percentile(solve, 50) * 1e3), "solve_ms_p99": float(np.percentile(solve, 99) * 1e3),
        "cold_latency_ms_p50": float(np.percentile(cold_lat, 50) * 1e3),
        "cold_latency_ms_max": float(cold_lat.max() * 1e3), "cold_pass_s": cold_wall,
        "all_converged": ok, "saturation_req_per_s": sat_rate,
        "saturation_mean_batch": float(np.mean(sat_batch)), "saturation_max_batch": int(max(sat_batch)),
        "poisson_mean_batch": float(np.mean([r["batch"] for *_, r in out])),
        "saturation_grouped_requests": int(sat_group),
        "poisson_grouped_requests": int(sum(r["group"] > 1 for *_, r in out)),
    }


def group_bench(args):
    """Grouped V-cycles: G problems of one lattice shape (3-D, Q2, 4 levels to
    32^3 cells; ellipsoids and unions of two from workloads.shape_family), FP32
    multigrid in FP64 CG to 1e-8 as in the solve server.  The G solves one
    after another (cmg_solve_multi with one column each, every V-cycle a graph
    replay) against one grouped solve (cmg_group_solve: every V-cycle step one
    launch over all G problems); the results must be identical."""
    import torch

    import workloads as W
    from paper_2508_11608_amd import Group, Problem

    ws = W.shape_family(args.group, seed=0)
    ps = [Problem(w) for w in ws]
    for p in ps:
        p.set_precision(True)
    bs = [torch.from_numpy(p.rhs_manufactured()).cuda() for p in ps]
    g = Group(ps)

    def alone():
        return [p.solve_multi(b[None, :], rtol=1e-8, maxit=200) for p, b in zip(ps, bs)]

    def grouped():
        return g.solve(bs, rtol=1e-8, maxit=200)

    def vc_alone():
        return [p.vcycle_multi(b[None, :]) for p, b in zip(ps, bs)]

    def vc_grouped():
        return g.vcycle(bs)

    def timed(f, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            out = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, out

    for _ in range(max(1, args.warmup)):
        alone()
        grouped()
        vc_alone()
        vc_grouped()
    t_alone, ra = timed(alone, args.steps)
    t_group, (xs, infos) = timed(grouped, args.steps)
    tv_alone, _ = timed(vc_alone, 10 * args.steps)
    tv_group, _ = timed(vc_grouped, 10 * args.steps)
    same = all(np.array_equal(x.cpu().numpy(), a[0][0].cpu().numpy()) and i["iterations"] == a[1][0]["iterations"]
               for x, i, a in zip(xs, infos, ra))
    nd = [p.ndofs() for p in ps]
    dofs = sum(n * i["iterations"] for n, i in zip(nd, infos))
    g.close()
    for p in ps:
        p.close()
    return {
        "metric": "grouped V-cycles: aggregate DoF/s per CG iteration", "value": dofs / t_group,
        "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_group * 1e3, "higher_is_better": True, "dtype": "f32 multigrid in f64 CG",
        "data": "synthetic",
        "config": {"workload": f"{len(ws)} problems of one lattice shape: 3-D, Q2, 4 levels to 32^3 cells, "
                               "ellipsoids and unions of two (workloads.shape_family seed 0), manufactured f, "
                               "rtol 1e-8",
                   "members": [w.name for w in ws], "n_dofs": nd,
                   "iterations": [int(i["iterations"]) for i in infos]},
        "alone_value": dofs / t_alone, "solve_ms_alone": t_alone * 1e3, "solve_ms_grouped": t_group * 1e3,
        "speedup": t_alone / t_group, "vcycle_ms_alone": tv_alone * 1e3, "vcycle_ms_grouped": tv_group * 1e3,
        "identical_to_alone": bool(same), "all_converged": all(i["status"] == 0 for i in infos),
    }


def paper_tables(args):
    """GMRES (restart 30) and the stand-alone V-cycle to 1e-9 on the paper's
    circle protocol, FP64, manufactured right-hand side, k = 1..3, n_c = 1..4,
    finest levels L from --paper-tables; the paper's printed counts from
    tests/golden/paper_iteration_tables.txt beside them."""
    import torch

    import workloads as W
    from paper_2508_11608_amd import Problem

    paper = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_iteration_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        solver, k, nc, L, it = line.split()
        paper[(solver, int(k), int(nc), int(L))] = None if it == "-" else int(it)
    rows = []
    t0 = time.perf_counter()
    for L in [int(v) for v in args.paper_tables.split(",")]:
        for k in (1, 2, 3):
            for nc in (1, 2, 3, 4):
                w = W.paper_circle(k, L, nc)
                P = Problem(w)
                b = torch.from_numpy(P.rhs_manufactured()).cuda()
                x = torch.empty_like(b)
                res = {}
                for solver in ("gmres", "vcycle"):
                    ts = time.perf_counter()
                    if solver == "gmres":
                        _, info = P.gmres(b, x, rtol=1e-9, maxit=500, restart=30, raise_on_fail=False)
                    else:
                        _, info = P.vcycle_solve(b, x, rtol=1e-9, maxit=500, raise_on_fail=False)
                    torch.cuda.synchronize()
                    res[solver] = (info["iterations"] if info["status"] == 0 else None, time.perf_counter() - ts)
                row = {"L": L, "k": k, "n_c": nc, "dofs": P.ndofs(),
                       "gmres": res["gmres"][0], "gmres_paper": paper.get(("gmres", k, nc, L)),
                       "vcycle": res["vcycle"][0], "vcycle_paper": paper.get(("vcycle", k, nc, L)),
                       "gmres_s": res["gmres"][1], "vcycle_s": res["vcycle"][1]}
                rows.append(row)
                print(f"[paper-tables] L={L} Q{k} n_c={nc}: {row['dofs']} DoFs, GMRES {row['gmres']} "
                      f"(paper {row['gmres_paper']}), V-cycle {row['vcycle']} (paper {row['vcycle_paper']}), "
                      f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
                P.close()
    return {"paper_tables": rows}


def ghost_sweep(args):
    """The paper's ghost-penalty study on its circle protocol (GMRES with the
    FP64 V-cycle to 1e-9, n_c = 2): for Q1 gamma_1 runs over 0.05..0.15 and the
    value with the smallest mean fractional count over the levels is kept; Q2
    then varies gamma_2 with that gamma_1, and Q3 gamma_3 with both earlier
    optima.  n_frac = n_it * 8 / -log10(||r_n|| / ||r_0||), the paper's
    formula.  The paper's printed values (tests/golden/paper_ghost_tables.txt)
    are reported beside ours."""
    import math

    import torch

    import workloads as W
    from paper_2508_11608_amd import Problem

    paper = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_ghost_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, L, g, v = line.split()
        paper[(int(k), int(L), g)] = float(v)
    Ls = [int(v) for v in args.ghost_sweep.split(",")]
    gammas = [round(0.05 + 0.01 * i, 2) for i in range(11)]
    rows, optimum = [], []
    t0 = time.perf_counter()
    for k in (1, 2, 3):
        mean = {}
        for g in gammas:
            gm = tuple(optimum) + (g,)
            acc = []
            for L in Ls:
                base = W.paper_circle(k, L)
                w = W.Workload(**{**base.__dict__, "gamma_m": gm, "name": f"{base.name}-g{gm}"})
                P = Problem(w)
                b = torch.from_numpy(P.rhs_manufactured()).cuda()
                _, info = P.gmres(b, rtol=1e-9, maxit=500, restart=30, raise_on_fail=False)
                P.close()
                nfrac = info["iterations"] * 8.0 / -math.log10(info["rel_residual"])
                acc.append(nfrac)
                rows.append({"k": k, "L": L, "gamma": g, "gamma_m": list(gm), "iterations": info["iterations"],
                             "n_frac": nfrac, "n_frac_paper": paper.get((k, L, f"{g:.2f}"))})
                print(f"[ghost-sweep] Q{k} L={L} gamma_m={gm}: {info['iterations']} its, n_frac {nfrac:.2f} "
                      f"(paper {rows[-1]['n_frac_paper']}), {time.perf_counter() - t0:.0f} s", file=sys.stderr,
                      flush=True)
            mean[g] = sum(acc) / len(acc)
        optimum.append(min(gammas, key=lambda g: (mean[g], g)))
    return {"ghost_sweep": rows, "optimum_gamma_m": optimum}


def kernel_source_hash() -> str:
    src = os.path.join(ROOT, "paper_2508_11608_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def algorithmic_bytes(P, w, kind: str, s: int = 8, m: int = 1, two_buffer: bool = True,
                      dense: bool = False) -> dict:
    """Algorithmic HBM bytes of every launch of one kernel kind in one V-cycle,
    keyed by (level, colour) (or level for 'apply'); s = 8 B (FP64 multigrid)
    or 4 B (FP32 multigrid), indices 4 B.  With m columns the matrix and index
    terms count once and the vector terms m times (shown for m = 1 below).

    interior_step, per patch:  s [(2k)^d + 2 (2k-1)^d] + 4
        x over the patch closure (same-coloured closures tile space with period
        2k nodes), b on the internal nodes, x written on them, vertex index.
    cut_solve, per patch j:    s N_j^2 + N_j (4 + 2 s) + 12 + s (2k)^d
                               + s k^d (k+1)^d x (cut cells of the patch)
        dense inverse, node list, b and the new x, offsets, x over the
        closure, and the k^d rows of every cut-cell matrix that belong to
        internal nodes of the patch; plus the copy blocks of a two-buffer step
        after colour p: 5 B (node, flag) per DoF of p and 2 s per DoF of p
        that the current colour does not own (every step of a pass but the
        first, in both passes; averaged over the colour's launches).
    apply (residual), per DoF: 4 + 3 s, plus s (k+1)^d ((k+1)^d + 1) / 2 per
        cut cell (its packed symmetric matrix); the CG product A p once per
        iteration on the finest level, always FP64: 4 + 2*8 per DoF plus the
        packed matrix in FP64 per cut cell.
    dense=True gives the operator terms for dense cut-cell matrices ((k+1)^{2d}
    per cut cell).
    """
    d, k = w.dim, w.k
    nl = (k + 1) ** d
    ncm = nl * nl if dense else nl * (nl + 1) // 2  # entries read per cut-cell matrix
    out = {}
    for l in range(1, w.n_levels):
        c = P.counts(l)
        if kind == "apply":
            out[l] = c["n_dofs"] * (4 + 3 * s * m) + c["cut_cells"] * ncm * s
            if l == w.n_levels - 1:  # the CG product A p on the finest level (no b)
                out["cg"] = c["n_dofs"] * (4 + 2 * 8 * m) + c["cut_cells"] * ncm * 8
            continue
        N = P.export(l, 2, np.uint8)  # cell flags, x fastest
        Nc = round(len(N) ** (1.0 / d))
        flags = N.reshape((Nc,) * d)  # index order (z, y, x) / (y, x)
        cut = (flags & 2) != 0
        copy = {}
        if kind == "cut_solve" and two_buffer:  # (the multi-column steps have no copy blocks)
            nodes = {c: P.export(l, 32 + c, np.int32) for c in range(2 ** d)}
            present = [c for c in range(2 ** d) if len(nodes[c])]
            for i, c in enumerate(present):
                total = 0
                for prev in (present[i - 1], present[(i + 1) % len(present)]):  # forward, backward pass
                    first = (prev == present[-1] and c == present[0]) or (prev == present[0] and c == present[-1])
                    times = w.n_c - 1 if (first and len(present) > 1) else w.n_c
                    if len(present) == 1:
                        times = w.n_c - 1
                    moved = np.count_nonzero(~np.isin(nodes[prev], nodes[c]))
                    total += times * (5 * len(nodes[prev]) + 2 * s * m * moved)
                copy[c] = total / (2 * w.n_c)
        for col in range(2 ** d):
            if kind == "interior_step":
                nv = len(P.export(l, 16 + col, np.int32))
                if nv:
                    out[(l, col)] = nv * (s * m * ((2 * k) ** d + 2 * (2 * k - 1) ** d) + 4)
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
            b = (s * nj ** 2 + nj * (4 + 2 * s * m) + 12 + s * m * (2 * k) ** d + s * k ** d * nl * ncut).sum()
            out[(l, col)] = int(b + copy.get(col, 0))
    return out


def vcycle_bytes(P, w, s: int = 8, m: int = 1, dense: bool = False) -> int:
    """Algorithmic bytes of one whole V-cycle (one pre- and one post-smoothing
    step per level, n_c sweeps over the cut colours):
        sum_{l >= 1} [2 (S_int + n_c S_cut) + R + T] + s (n_0^2 + 2 n_0)
    with S_int / S_cut the interior / cut colour steps of a sweep (per patch as
    in algorithmic_bytes, copy blocks of the two-buffer steps included), R the
    level residual b - A x, T the transfers s (3 n_l + 2 n_{l-1}) (prolongation
    reads e and x and writes x, restriction reads r and writes the coarse b),
    and the coarse solve a GEMV with the dense inverse.  With m columns the
    matrix terms count once; dense as in algorithmic_bytes."""
    inter = algorithmic_bytes(P, w, "interior_step", s, m)
    cut = algorithmic_bytes(P, w, "cut_solve", s, m, two_buffer=(m == 1))
    app = algorithmic_bytes(P, w, "apply", s, m, dense=dense)
    total = 2 * sum(inter.values()) + 2 * w.n_c * sum(cut.values())
    total += sum(v for key, v in app.items() if key != "cg")
    n = [P.counts(l)["n_dofs"] for l in range(w.n_levels)]
    for l in range(1, w.n_levels):
        total += s * m * (3 * n[l] + 2 * n[l - 1])
    total += s * n[0] * n[0] + 2 * s * m * n[0]
    return int(total)


def roofline(P, w, kind: str, launches: int, total_ms: float, vcycles: int, fp32: bool = False,
             ncol: int = 1, two_buffer: bool = True, level: int = None) -> dict:
    """Live roofline of one kernel kind: algorithmic bytes per launch over the
    average HIP-event duration of its launches, on one level (the launches
    timed) or on all of them."""
    per_v = algorithmic_bytes(P, w, kind, 4 if fp32 else 8, ncol, two_buffer)
    if level is not None:
        per_v = {key: v for key, v in per_v.items()
                 if (key[0] if isinstance(key, tuple) else (w.n_levels - 1 if key == "cg" else key)) == level}
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
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kind}_{'fp32' if fp32 else 'fp64'}_{w.name}.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("kernel_source_sha256_16") == kernel_source_hash():
            traffic = t.get("bytes_per_launch")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kind,
            "level": "all" if level is None else level,
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


def timed_multi_solves(P, w, B, args, fp32: bool) -> dict:
    """Multi-column variant: args.steps solves of all columns of B at once
    (independent PCG per column sharing multi-column V-cycles).  value counts
    DoFs x columns x V-cycle applications per second."""
    import torch

    P.set_precision(fp32)
    n = P.ndofs()
    nrhs = B.shape[0]
    X = torch.empty_like(B)
    for _ in range(args.warmup):
        P.solve_multi(B, X, rtol=1e-8)
    torch.cuda.synchronize()
    fine = w.n_levels - 1
    P.timing([args.kernel], level=fine)
    vcyc = 0
    lat = []
    infos = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, infos = P.solve_multi(B, X, rtol=1e-8)
        lat.append(time.perf_counter() - ts)
        vcyc += max(i["iterations"] for i in infos)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms = P.timing_read(args.kernel, fine)
    P.timing([])
    roof = roofline(P, w, args.kernel, launches, kms, vcyc, fp32, ncol=nrhs, two_buffer=False, level=fine)
    tag = "fp32" if fp32 else "fp64"
    print(f"[bench] {tag} x{nrhs}: timed {args.steps} solves: {dt:.3f}s, {vcyc} multi V-cycles", file=sys.stderr,
          flush=True)
    R = torch.randn(B.shape, dtype=torch.float64, device="cuda")
    Z = torch.empty_like(R)
    for _ in range(2):
        P.vcycle_multi(R, Z)
    torch.cuda.synchronize()
    nv = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(nv):
        P.vcycle_multi(R, Z)
    e1.record()
    torch.cuda.synchronize()
    t_v = e0.elapsed_time(e1) / 1e3 / nv
    bv = vcycle_bytes(P, w, 4 if fp32 else 8, nrhs)
    bv_dense = vcycle_bytes(P, w, 4 if fp32 else 8, nrhs, dense=True)
    vroof = {"bound": "hbm", "algorithmic_bytes": bv, "vcycle_ms": t_v * 1e3, "achieved": bv / t_v / 1e9,
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bv / t_v / 1e9 / HBM_PEAK_GBS,
             "algorithmic_bytes_dense_storage": bv_dense}
    return {"precision": "fp32 multigrid, fp64 CG" if fp32 else "fp64", "value": n * nrhs * vcyc / dt,
            "x": X.clone(), "vcycle_roofline": vroof,
            "ms_per_step": dt / args.steps * 1e3, "iterations_per_column": [i["iterations"] for i in infos],
            "final_rel_residual": max(i["rel_residual"] for i in infos),
            "solve_latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "solve_latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "vcycle_ms": t_v * 1e3, "vcycle_dofs_per_s": n * nrhs / t_v, "roofline": roof}


def timed_solves(P, w, b, x, args, fp32: bool) -> dict:
    """Warm-up, then args.steps timed solves in one precision of the multigrid
    (CG is FP64 either way), the live roofline of args.kernel, and back-to-back
    V-cycles timed separately outside the timed region."""
    import torch

    P.set_precision(fp32)
    n = P.ndofs()
    for _ in range(args.warmup):
        P.solve(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    fine = w.n_levels - 1
    P.timing([args.kernel], level=fine)  # the finest level's launches only: few events, no host stall
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
    launches, kms = P.timing_read(args.kernel, fine)
    P.timing([])
    roof = roofline(P, w, args.kernel, launches, kms, its, fp32, level=fine)
    tag = "fp32" if fp32 else "fp64"
    print(f"[bench] {tag}: timed {args.steps} solves: {dt:.3f}s, {its} V-cycles", file=sys.stderr, flush=True)
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
    bv = vcycle_bytes(P, w, 4 if fp32 else 8)
    bv_dense = vcycle_bytes(P, w, 4 if fp32 else 8, dense=True)
    vroof = {"bound": "hbm", "algorithmic_bytes": bv, "vcycle_ms": t_v * 1e3, "achieved": bv / t_v / 1e9,
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bv / t_v / 1e9 / HBM_PEAK_GBS,
             "algorithmic_bytes_dense_storage": bv_dense}
    return {"precision": "fp32 multigrid, fp64 CG" if fp32 else "fp64", "value": n * its / dt,
            "x": x.clone(), "vcycle_roofline": vroof,
            "ms_per_step": dt / args.steps * 1e3, "iterations_per_solve": its / args.steps,
            "final_rel_residual": rel,
            "solve_latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "solve_latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "vcycle_ms": t_v * 1e3, "vcycle_dofs_per_s": n / t_v, "roofline": roof}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU decomposition is a design note, "
              "not an implementation", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.serve:
        torch.cuda.set_device(0)
        print(json.dumps(serve(args)), flush=True)
        return
    if args.group:
        torch.cuda.set_device(0)
        print(json.dumps(group_bench(args)), flush=True)
        return
    if args.ghost_sweep:
        torch.cuda.set_device(0)
        print(json.dumps(ghost_sweep(args)), flush=True)
        return
    if args.paper_tables:
        torch.cuda.set_device(0)
        print(json.dumps(paper_tables(args)), flush=True)
        return

    import workloads as W
    from paper_2508_11608_amd import Problem

    w = {"ball": W.ball_q2, "disc": W.disc_q2, "union8": W.sphere_union_8}[args.workload]()
    if args.levels:
        w = w.with_levels(args.levels)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    P = Problem(w)
    t_setup = time.perf_counter() - t0
    if args.no_graphs:
        P.set_graphs(False)
    if args.small_cut_launch is not None:
        P.set_launch(args.small_cut_launch, 2048)
    n = P.ndofs()
    print(f"[bench] {w.name}: {n} DoFs, setup {t_setup:.1f}s", file=sys.stderr, flush=True)
    b = torch.from_numpy(P.rhs_manufactured()).cuda()
    x = torch.empty_like(b)
    first = [True, False] if args.fp32 else [False, True]
    if args.nrhs > 1:
        if args.nrhs > 8:
            raise SystemExit("at most 8 right-hand sides")
        B = torch.from_numpy(np.stack([P.rhs_fourier(*W.fourier_modes(w.dim, seed=1000 + c))
                                       for c in range(args.nrhs)])).cuda()
        res = {fp32: timed_multi_solves(P, w, B, args, fp32) for fp32 in first}
    else:
        res = {fp32: timed_solves(P, w, b, x, args, fp32) for fp32 in first}
    # error of every result against the FP64 reference: the FP64 multigrid in
    # FP64 CG driven to 1e-12 on the same right-hand sides (the FP64 GPU path,
    # which the parity tests tie to the CPU oracle; the oracle itself does not
    # run at this size)
    P.set_precision(False)
    if args.nrhs > 1:
        xref = torch.empty_like(B)
        _, iref = P.solve_multi(B, xref, rtol=1e-12, maxit=400, raise_on_fail=False)
        ref_note = f"FP64 multigrid + FP64 CG to 1e-12 ({max(i['iterations'] for i in iref)} iterations)"
    else:
        xref = torch.empty_like(b)
        _, iref = P.solve(b, xref, rtol=1e-12, maxit=400, raise_on_fail=False)
        ref_note = f"FP64 multigrid + FP64 CG to 1e-12 ({iref['iterations']} iterations)"
    xs = {fp32: res[fp32].pop("x") for fp32 in first}
    for fp32 in first:
        res[fp32]["error_vs_fp64_reference"] = float(torch.linalg.norm(xs[fp32] - xref) / torch.linalg.norm(xref))
        res[fp32]["fp64_reference"] = ref_note
    # the FP32-preconditioned solution against the FP64-preconditioned one at the same tolerance
    res[True]["diff_vs_fp64_solve_same_rtol"] = float(torch.linalg.norm(xs[True] - xs[False])
                                                      / torch.linalg.norm(xs[False]))
    head = res[first[0]]
    other = res[first[1]]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DoF/s" if args.nrhs == 1 else "DoF*rhs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 multigrid in f64 CG" if args.fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {DOMAINS[args.workload]} in [-1,1]^{w.dim}, Q{w.k}, {w.n_levels} "
                               f"levels to {w.fine_cells}^{w.dim} cells, "
                               + (f"{args.nrhs} seeded Fourier right-hand sides per solve (independent PCG per "
                                  f"column, shared multi-column V-cycles)" if args.nrhs > 1 else "manufactured f")
                               + ", FP64 CG to 1e-8",
                   "active_dofs": n, "n_c": w.n_c, "nrhs": args.nrhs, "vcycle_graphs": not args.no_graphs,
                   "precision": "fp32 preconditioner, fp64 CG" if args.fp32 else "fp64"},
        "roofline": head["roofline"],
        "cg_iterations_per_solve": head.get("iterations_per_solve", head.get("iterations_per_column")),
        "final_rel_residual": head["final_rel_residual"],
        "solve_latency_ms_p50": head["solve_latency_ms_p50"],
        "solve_latency_ms_p99": head["solve_latency_ms_p99"],
        "vcycle_ms": head["vcycle_ms"],
        "vcycle_dofs_per_s": head["vcycle_dofs_per_s"],
        "vcycle_roofline": head["vcycle_roofline"],
        "error_vs_fp64_reference": head["error_vs_fp64_reference"],
        "fp64_reference": head["fp64_reference"],
        "setup_s": t_setup,
        ("fp64" if args.fp32 else "fp32_precond"): other,
    }
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
