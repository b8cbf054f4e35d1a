"""HIP path vs the CPU oracle, element by element, through the C ABI.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.disc_q2(), W.offcentre_disc(1, 4), W.offcentre_disc(3, 3), W.ellipse(2, 3),
         W.offcentre_ball(2, 3), W.ball_q2().with_levels(3), W.offcentre_ball(3, 2), W.offcentre_ball(1, 3),
         W.disc_union(2, 3), W.ball_union(2, 3), W.box_disc(1, 4), W.box_disc(2, 4), W.box_disc(3, 3),
         W.box_ball(2, 3),
         W.Workload(**{**W.offcentre_disc(3, 3).__dict__, "name": "disc-off-Q3-gamma-m", "gamma_m": (0.07, 0.12, 0.05)})]

TOL_APPLY = 1e-12
TOL_SMOOTH = 1e-11
TOL_VCYCLE = 1e-10


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    import torch
    from oracle import problem as OP
    from paper_2508_11608_amd import Problem

    w = request.param
    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels}", flush=True)
    P = Problem(w)
    levels, mats, prols, H = OP.build(w)
    yield w, P, levels, mats, prols, H
    P.close()
    torch.cuda.synchronize()


def _cuda(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_apply_every_level(case):
    w, P, levels, mats, _, _ = case
    for l in range(len(levels)):
        x = W.random_vector(levels[l].n_dofs, seed=10 + l)
        y = P.apply(l, _cuda(x)).cpu().numpy()
        assert _rel(y, mats[l] @ x) < TOL_APPLY, l


def test_colour_steps(case):
    w, P, levels, mats, _, H = case
    for l in range(1, len(levels)):
        n = levels[l].n_dofs
        b = W.random_vector(n, seed=20 + l)
        x0 = W.random_vector(n, seed=30 + l)
        for key in H.schedule(l)[: 2 * 2 ** w.dim]:
            xr = x0.copy()
            H.colour_step(l, key, xr, b)
            xg = _cuda(x0)
            P.colour_step(l, key[0], key[1], xg, _cuda(b))
            assert _rel(xg.cpu().numpy(), xr) < TOL_SMOOTH, (l, key)


def test_smoother_pre_and_post(case):
    w, P, levels, _, _, H = case
    l = len(levels) - 1
    n = levels[l].n_dofs
    b = W.random_vector(n, seed=41)
    for post in (False, True):
        x0 = W.random_vector(n, seed=42 + post)
        xr = x0.copy()
        H.smooth(l, xr, b, post=post)
        xg = _cuda(x0)
        P.smooth(l, post, xg, _cuda(b))
        assert _rel(xg.cpu().numpy(), xr) < TOL_SMOOTH, post


def test_transfers(case):
    w, P, levels, _, prols, _ = case
    for l in range(1, len(levels)):
        xc = W.random_vector(levels[l - 1].n_dofs, seed=50 + l)
        xf = W.random_vector(levels[l].n_dofs, seed=60 + l)
        assert _rel(P.prolongate(l, _cuda(xc)).cpu().numpy(), prols[l - 1] @ xc) < 1e-14
        assert _rel(P.restrict(l, _cuda(xf)).cpu().numpy(), prols[l - 1].T @ xf) < 1e-14


def test_coarse_solve(case):
    w, P, levels, mats, _, _ = case
    b = W.random_vector(levels[0].n_dofs, seed=70)
    x = P.coarse_solve(_cuda(b)).cpu().numpy()
    assert _rel(x, np.linalg.solve(mats[0].toarray(), b)) < 1e-10


def test_vcycle(case):
    w, P, levels, _, _, H = case
    r = W.random_vector(levels[-1].n_dofs, seed=80)
    z = P.vcycle(_cuda(r)).cpu().numpy()
    assert _rel(z, H.vcycle(r)) < TOL_VCYCLE


def test_vcycle_deterministic(case):
    w, P, levels, _, _, _ = case
    r = _cuda(W.random_vector(levels[-1].n_dofs, seed=81))
    z1 = P.vcycle(r).cpu().numpy()
    z2 = P.vcycle(r).cpu().numpy()
    assert np.array_equal(z1, z2)


def test_pcg_solve(case):
    from oracle import problem as OP
    from oracle.multigrid import pcg

    w, P, levels, mats, _, H = case
    b = P.rhs_manufactured()
    x, info = P.solve(_cuda(b), rtol=1e-8, maxit=300)
    xr, it, _ = pcg(mats[-1], OP.rhs(w, levels[-1]), H.vcycle, rtol=1e-8, maxit=300)
    assert abs(info["iterations"] - it) <= 1
    assert info["rel_residual"] <= 1e-8
    # the same iterates up to rounding when the counts agree; one more or less
    # iteration moves the iterate by up to the tolerance
    err = _rel(x.cpu().numpy(), xr)
    print(f"  PCG: {info['iterations']} its (oracle {it}), solution rel diff {err:.2e}")
    assert err < (1e-10 if info["iterations"] == it else 1e-8)


# ---- mixed precision: FP32 multigrid inside FP64 CG --------------------------
# FP32 results are compared with the oracle run in float32 (same definition,
# different summation order).  The tolerance is tied to the size of the FP32
# effect itself: 10x the oracle's own float32-vs-float64 deviation (+1e-6).

_H32 = {}


@pytest.fixture
def fp32_case(case):
    """The case with the library switched to the FP32 multigrid for one test."""
    from oracle.multigrid import Hierarchy

    w, P, levels, mats, prols, H = case
    if w.name not in _H32:
        _H32[w.name] = Hierarchy(levels, mats, prols, n_c=w.n_c, dtype=np.float32)
    P.set_precision(True)
    try:
        yield w, P, levels, mats, prols, H, _H32[w.name]
    finally:
        P.set_precision(False)


def _tol32(ref32, ref64):
    return 10.0 * _rel(ref32, ref64) + 1e-6


def test_fp32_apply_and_transfers(fp32_case):
    w, P, levels, mats, prols, H, H32 = fp32_case
    l = len(levels) - 1
    x = W.random_vector(levels[l].n_dofs, seed=90)
    y64 = mats[l] @ x
    y32 = (H32.A[l] @ x.astype(np.float32)).astype(np.float64)
    assert _rel(P.apply(l, _cuda(x)).cpu().numpy(), y32) < _tol32(y32, y64)
    xc = W.random_vector(levels[l - 1].n_dofs, seed=91)
    p64 = prols[l - 1] @ xc
    p32 = (H32.P[l] @ xc.astype(np.float32)).astype(np.float64)
    assert _rel(P.prolongate(l, _cuda(xc)).cpu().numpy(), p32) < _tol32(p32, p64)


def test_fp32_smoother(fp32_case):
    w, P, levels, mats, prols, H, H32 = fp32_case
    l = len(levels) - 1
    n = levels[l].n_dofs
    b = W.random_vector(n, seed=92)
    x0 = W.random_vector(n, seed=93)
    x64 = x0.copy()
    H.smooth(l, x64, b)
    x32 = x0.astype(np.float32)
    H32.smooth(l, x32, b.astype(np.float32))
    xg = _cuda(x0)
    P.smooth(l, False, xg, _cuda(b))
    x32 = x32.astype(np.float64)
    assert _rel(xg.cpu().numpy(), x32) < _tol32(x32, x64)


def test_fp32_vcycle(fp32_case):
    w, P, levels, mats, prols, H, H32 = fp32_case
    r = W.random_vector(levels[-1].n_dofs, seed=94)
    z64 = H.vcycle(r)
    z32 = H32.vcycle(r).astype(np.float64)
    zg = P.vcycle(_cuda(r)).cpu().numpy()
    print(f"  fp32 V-cycle: oracle32 vs 64 {_rel(z32, z64):.2e}, gpu32 vs oracle32 {_rel(zg, z32):.2e}")
    assert _rel(zg, z32) < _tol32(z32, z64)


def test_fp32_pcg(fp32_case):
    from oracle import problem as OP
    from oracle.multigrid import pcg

    w, P, levels, mats, prols, H, H32 = fp32_case
    b = P.rhs_manufactured()
    x, info = P.solve(_cuda(b), rtol=1e-8, maxit=300)
    bo = OP.rhs(w, levels[-1])
    x64, it64, _ = pcg(mats[-1], bo, H.vcycle, rtol=1e-8, maxit=300)
    _, it32, _ = pcg(mats[-1], bo, H32.vcycle, rtol=1e-8, maxit=300)
    err = _rel(x.cpu().numpy(), x64)
    print(f"  fp32-preconditioned CG: {info['iterations']} its (oracle fp32 {it32}, fp64 {it64}), "
          f"rel residual {info['rel_residual']:.2e}, error vs FP64 oracle solution {err:.2e}")
    assert abs(info["iterations"] - it32) <= 1
    assert info["rel_residual"] <= 1e-8
    assert err < 1e-6
