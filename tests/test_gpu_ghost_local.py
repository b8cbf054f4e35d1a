"""Cut colour steps with the patch-local residual (x beyond a patch's closure
taken as zero, cmg_set_ghost_coupling(1)) through the C ABI against the oracle's
variant: colour steps, smoothers and V-cycle per level, GMRES iteration counts;
CG and the multi-column calls refuse the variant.  Both ghost-face code paths of
the cut-patch kernel are covered: the FP64 Q2 3-D kernel, which stages the
halo slabs in LDS, and the others, which read the face nodes from memory.

Every case prints its name first so that a failing GPU run can be located."""
import copy

import numpy as np
import pytest

import oracle_cache
import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.offcentre_disc(2, 4), W.offcentre_disc(3, 3), W.offcentre_ball(2, 3), W.ball_union(2, 3),
         W.offcentre_ball(1, 3)]


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    import torch
    from paper_2508_11608_amd import Problem

    w = request.param
    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} (patch-local ghost coupling)", flush=True)
    P = Problem(w)
    P.set_ghost_coupling(True)
    levels, mats, prols, H = oracle_cache.build(w)
    Hl = copy.copy(H)
    Hl.ghost_local = True
    yield w, P, levels, mats, H, Hl
    P.close()
    torch.cuda.synchronize()


def _cuda(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_colour_steps_and_smoothers(case):
    w, P, levels, mats, H, Hl = case
    for l in range(1, len(levels)):
        n = levels[l].n_dofs
        b = W.random_vector(n, seed=600 + l)
        x0 = W.random_vector(n, seed=610 + l)
        for key in Hl.schedule(l):
            if key[0]:
                continue
            xr = x0.copy()
            Hl.colour_step(l, key, xr, b)
            xg = _cuda(x0)
            P.colour_step(l, key[0], key[1], xg, _cuda(b))
            assert _rel(xg.cpu().numpy(), xr) < 1e-11, (l, key)
        for post in (False, True):
            xr = x0.copy()
            Hl.smooth(l, xr, b, post=post)
            xg = _cuda(x0)
            P.smooth(l, post, xg, _cuda(b))
            assert _rel(xg.cpu().numpy(), xr) < 1e-11, (l, post)


def test_vcycle_and_inconsistency(case):
    """V-cycle parity, and the variant differs from the exact one by about as
    much on the GPU as in the oracle (the measured inconsistency)."""
    w, P, levels, mats, H, Hl = case
    r = W.random_vector(levels[-1].n_dofs, seed=620)
    zl = P.vcycle(_cuda(r)).cpu().numpy()
    zr = Hl.vcycle(r)
    assert _rel(zl, zr) < 1e-10
    P.set_ghost_coupling(False)
    try:
        ze = P.vcycle(_cuda(r)).cpu().numpy()
    finally:
        P.set_ghost_coupling(True)
    d_gpu, d_ora = _rel(zl, ze), _rel(zr, H.vcycle(r))
    print(f"  V-cycle: parity {_rel(zl, zr):.2e}; patch-local vs exact {d_gpu:.3e} (oracle {d_ora:.3e})")
    assert abs(d_gpu - d_ora) <= 1e-6 * max(d_ora, 1e-300) + 1e-12


def test_gmres(case):
    """GMRES with the variant as preconditioner, 2-D cases: iteration counts
    within +-1 of the oracle.  (In 3-D the oracle's GMRES(30) with this variant
    stalls: the dropped ghost terms reach the ill-conditioned cut-patch solves,
    so one smoothing step moves the discrete solution by O(1); running it to
    maxit in the oracle takes minutes, so 3-D is left to the V-cycle parity.)"""
    from oracle import problem as OP
    from oracle.multigrid import gmres

    w, P, levels, mats, H, Hl = case
    if w.dim != 2:
        pytest.skip("3-D: the variant's GMRES stalls in the oracle too (V-cycle parity covers it)")
    b = OP.rhs(w, levels[-1])
    x, info = P.gmres(_cuda(b), rtol=1e-9, maxit=300, restart=30)
    xr, it, _ = gmres(mats[-1], b, Hl.vcycle, rtol=1e-9, restart=30, maxit=300)
    _, it_exact, _ = gmres(mats[-1], b, H.vcycle, rtol=1e-9, restart=30, maxit=300)
    print(f"  GMRES: patch-local {info['iterations']} its (oracle {it}), exact coupling (oracle) {it_exact}")
    assert abs(info["iterations"] - it) <= 1
    assert np.linalg.norm(b - mats[-1] @ x.cpu().numpy()) <= 1.01e-9 * np.linalg.norm(b)


def test_cg_and_multi_column_refuse_the_variant(case):
    from paper_2508_11608_amd import CutmgError

    w, P, levels, mats, H, Hl = case
    b = _cuda(W.random_vector(levels[-1].n_dofs, seed=630))
    for call in (lambda: P.solve(b), lambda: P.vcycle_multi(b.reshape(1, -1).contiguous())):
        with pytest.raises(CutmgError) as e:
            call()
        assert e.value.status == -1
