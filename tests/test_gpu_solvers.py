"""The paper's other outer solvers through the C ABI against the oracle:
right-preconditioned restarted GMRES (cmg_gmres) and the V-cycle as a
stand-alone solver (cmg_vcycle_solve), on the paper's circle protocol.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.paper_circle(1, 4), W.paper_circle(2, 4), W.paper_circle(3, 3), W.paper_circle(3, 3, n_c=1),
         W.offcentre_ball(2, 3)]


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    import torch
    from oracle import problem as OP
    from paper_2508_11608_amd import Problem

    w = request.param
    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} n_c={w.n_c} (outer solvers)", flush=True)
    P = Problem(w)
    levels, mats, prols, H = OP.build(w)
    b = P.rhs_manufactured()
    yield w, P, levels, mats, H, b
    P.close()
    torch.cuda.synchronize()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_gmres_matches_oracle(case):
    import torch
    from oracle.multigrid import gmres

    w, P, levels, mats, H, b = case
    x, info = P.gmres(torch.from_numpy(b).cuda(), rtol=1e-9, maxit=300, restart=30)
    xr, it, _ = gmres(mats[-1], b, H.vcycle, rtol=1e-9, restart=30, maxit=300)
    print(f"  GMRES: library {info['iterations']} its, oracle {it}")
    assert abs(info["iterations"] - it) <= 1
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - mats[-1] @ xg) <= 1.01e-9 * np.linalg.norm(b)
    assert _rel(xg, xr) < 1e-6


def test_vcycle_solver_matches_oracle(case):
    import torch
    from oracle.multigrid import vcycle_iteration

    w, P, levels, mats, H, b = case
    xr, it, hist = vcycle_iteration(mats[-1], b, H.vcycle, rtol=1e-9, maxit=400)
    x, info = P.vcycle_solve(torch.from_numpy(b).cuda(), rtol=1e-9, maxit=400, raise_on_fail=False)
    print(f"  V-cycle solver: library {info['iterations']} its (status {info['status']}), oracle {it}")
    if it is None:  # the oracle iteration diverges; so must the library's
        assert info["status"] == -5
        return
    assert info["status"] == 0
    assert abs(info["iterations"] - it) <= 1
    assert _rel(x.cpu().numpy(), xr) < 1e-6


def test_gmres_in_fp32_multigrid(case):
    """FP32 V-cycle inside FP64 GMRES reaches the same tolerance with at most
    one more iteration than the FP64 V-cycle."""
    import torch

    w, P, levels, mats, H, b = case
    bg = torch.from_numpy(b).cuda()
    _, i64 = P.gmres(bg, rtol=1e-9)
    P.set_precision(True)
    try:
        x, i32 = P.gmres(bg, rtol=1e-9)
    finally:
        P.set_precision(False)
    assert abs(i32["iterations"] - i64["iterations"]) <= 1
    assert np.linalg.norm(b - mats[-1] @ x.cpu().numpy()) <= 1.01e-9 * np.linalg.norm(b)


def test_cg_stopped_at_maxit_is_enotconv_with_the_last_iterate(case):
    """An unreachable tolerance with maxit = 2: CMG_ENOTCONV, two iterations
    reported, and x is the oracle's PCG iterate after two steps."""
    import torch
    from oracle.multigrid import pcg

    w, P, levels, mats, H, b = case
    x, info = P.solve(torch.from_numpy(b).cuda(), rtol=1e-15, maxit=2, raise_on_fail=False)
    xr, it, hist = pcg(mats[-1], b, H.vcycle, rtol=1e-15, maxit=2)
    print(f"  CG maxit 2: status {info['status']}, residual {info['rel_residual']:.3e} (oracle {hist[-1]:.3e})")
    assert info["status"] == -5 and info["iterations"] == 2 and it == 2
    assert abs(info["rel_residual"] - hist[-1]) <= 1e-8 * hist[-1]
    assert _rel(x.cpu().numpy(), xr) < 1e-8


def test_non_finite_right_hand_side_is_einval(case):
    """A NaN in b is refused before any iteration (CMG_EINVAL)."""
    import torch

    w, P, levels, mats, H, b = case
    bn = b.copy()
    bn[len(bn) // 2] = np.nan
    _, info = P.solve(torch.from_numpy(bn).cuda(), raise_on_fail=False)
    assert info["status"] == -1 and info["iterations"] == 0
