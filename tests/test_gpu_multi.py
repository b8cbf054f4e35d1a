"""Several right-hand sides at once (cmg_vcycle_multi / cmg_solve_multi) through
the C ABI: FP64 columns (cut-patch steps with every inverse read once for all
columns) match single-column runs to rounding and the oracle V-cycle to 1e-10;
FP32 columns (cut local solves on the matrix cores) match the float32 oracle
V-cycle per column; every column's result is independent of the other columns
bit for bit; the multi-column PCG keeps every column's iteration count.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.disc_q2(), W.offcentre_ball(3, 2), W.ball_union(2, 3)]


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    import torch
    from oracle import problem as OP
    from oracle.multigrid import Hierarchy
    from paper_2508_11608_amd import Problem

    w = request.param
    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} (multi-column)", flush=True)
    P = Problem(w)
    levels, mats, prols, H = OP.build(w)
    H32 = Hierarchy(levels, mats, prols, n_c=w.n_c, dtype=np.float32)
    yield w, P, levels, mats, H, H32
    P.close()
    torch.cuda.synchronize()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _cols(n, nrhs, seed):
    return np.stack([W.random_vector(n, seed=seed + c) for c in range(nrhs)])


@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_fp64_columns_match_single_vcycles_and_oracle(case, nrhs):
    import torch

    w, P, levels, mats, H, _ = case
    P.set_precision(False)
    rn = _cols(levels[-1].n_dofs, nrhs, 100)
    r = torch.from_numpy(rn).cuda()
    z = P.vcycle_multi(r).cpu().numpy()
    for c in range(nrhs):
        zc = P.vcycle(r[c].contiguous()).cpu().numpy()
        zo = H.vcycle(rn[c])
        print(f"  column {c}: multi vs single {_rel(z[c], zc):.2e}, multi vs oracle {_rel(z[c], zo):.2e}")
        assert _rel(z[c], zc) < 1e-11, c
        assert _rel(z[c], zo) < 1e-10, c


@pytest.mark.parametrize("nrhs", [1, 2, 8])
def test_fp32_columns_match_oracle(case, nrhs):
    """Matrix-core local solves: each column against the float32 oracle and
    against the FP64 V-cycle, with the FP32 tolerance of the single-column tests
    (10x the oracle's own float32-vs-float64 deviation + 1e-6)."""
    import torch

    w, P, levels, mats, H, H32 = case
    n = levels[-1].n_dofs
    rs = _cols(n, nrhs, 200)
    P.set_precision(True)
    try:
        z = P.vcycle_multi(torch.from_numpy(rs).cuda()).cpu().numpy()
        single = [P.vcycle(torch.from_numpy(rs[c]).cuda()).cpu().numpy() for c in range(nrhs)]
    finally:
        P.set_precision(False)
    for c in range(nrhs):
        z64 = H.vcycle(rs[c])
        z32 = H32.vcycle(rs[c]).astype(np.float64)
        tol = 10.0 * _rel(z32, z64) + 1e-6
        print(f"  column {c}: multi vs oracle32 {_rel(z[c], z32):.2e}, single vs oracle32 {_rel(single[c], z32):.2e},"
              f" multi vs fp64 {_rel(z[c], z64):.2e}, single vs fp64 {_rel(single[c], z64):.2e}")
        assert _rel(z[c], z32) < tol
        assert _rel(z[c], z64) < tol


def test_columns_do_not_depend_on_their_neighbours(case):
    """A column's result is the same, bit for bit, whatever other columns run
    with it (FP64 and FP32, the latter with matrix-core local solves also for
    one column)."""
    import torch

    w, P, levels, *_ = case
    rs = torch.from_numpy(_cols(levels[-1].n_dofs, 8, 300)).cuda()
    for fp32 in (False, True):
        P.set_precision(fp32)
        try:
            z8 = P.vcycle_multi(rs)
            z3 = P.vcycle_multi(rs[:3].contiguous())
            z1 = P.vcycle_multi(rs[2:3].contiguous())
        finally:
            P.set_precision(False)
        assert torch.equal(z8[:3], z3), fp32
        assert torch.equal(z8[2], z1[0]), fp32


def test_fp64_multi_solve_matches_single_solves(case):
    import torch

    w, P, levels, *_ = case
    P.set_precision(False)
    n = levels[-1].n_dofs
    kap = [W.fourier_modes(w.dim, seed=1000 + c) for c in range(3)]
    B = np.stack([P.rhs_manufactured()] + [P.rhs_fourier(*m) for m in kap[:2]] + [np.zeros(n)])
    X, infos = P.solve_multi(torch.from_numpy(B).cuda(), rtol=1e-8, maxit=300)
    assert infos[3]["iterations"] == 0  # zero right-hand side: x = 0 without iterating
    assert not X[3].any()
    for c in range(3):
        xc, info = P.solve(torch.from_numpy(B[c]).cuda(), rtol=1e-8, maxit=300)
        d = _rel(X[c].cpu().numpy(), xc.cpu().numpy())
        print(f"  column {c}: {infos[c]['iterations']} its (single {info['iterations']}), solution diff {d:.2e}")
        assert abs(infos[c]["iterations"] - info["iterations"]) <= 1, c
        assert infos[c]["rel_residual"] <= 1e-8
        if infos[c]["iterations"] == info["iterations"]:
            assert d < 1e-9, c


def test_fp32_multi_solve(case):
    """Eight Fourier right-hand sides, FP32 multigrid with matrix-core local
    solves inside FP64 CG: every column converges to 1e-8 within one
    iteration of its single-column FP32 solve, close to the FP64 solution."""
    import torch

    w, P, levels, *_ = case
    B = np.stack([P.rhs_fourier(*W.fourier_modes(w.dim, seed=1000 + c)) for c in range(8)])
    Bg = torch.from_numpy(B).cuda()
    P.set_precision(False)
    X64, _ = P.solve_multi(Bg, rtol=1e-10, maxit=300)
    P.set_precision(True)
    try:
        X, infos = P.solve_multi(Bg, rtol=1e-8, maxit=300)
        for c in range(8):
            _, info = P.solve(Bg[c].contiguous(), rtol=1e-8, maxit=300)
            err = _rel(X[c].cpu().numpy(), X64[c].cpu().numpy())
            print(f"  column {c}: {infos[c]['iterations']} its (single {info['iterations']}), "
                  f"rel residual {infos[c]['rel_residual']:.2e}, error vs FP64 solution {err:.2e}")
            assert abs(infos[c]["iterations"] - info["iterations"]) <= 1
            assert infos[c]["rel_residual"] <= 1e-8
            assert err < 1e-6
    finally:
        P.set_precision(False)


def test_bad_column_counts_are_rejected(case):
    import torch

    from paper_2508_11608_amd.cutmg import CutmgError

    w, P, levels, *_ = case
    n = levels[-1].n_dofs
    with pytest.raises(CutmgError):
        P.vcycle_multi(torch.zeros((9, n), dtype=torch.float64, device="cuda"))
    with pytest.raises(CutmgError):
        P.solve_multi(torch.zeros((9, n), dtype=torch.float64, device="cuda"))
