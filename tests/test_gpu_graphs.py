"""V-cycles replayed from captured HIP graphs (the default) against
kernel-by-kernel launches, through the C ABI: every replay equals the eager
result bit for bit, with the program's own eager work and synchronisations
between the replays, in both precisions, one and several columns, inside CG;
and kernel timing still counts every timed launch of every replay.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.disc_q2(), W.ball_q2().with_levels(3), W.ball_union(2, 3), W.offcentre_disc(3, 3)]


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    import torch
    from paper_2508_11608_amd import Problem

    w = request.param
    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} (graph replays)", flush=True)
    P = Problem(w)
    yield w, P
    P.close()
    torch.cuda.synchronize()


def _cuda(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_replays_equal_eager(case, fp32):
    import torch

    w, P = case
    n = P.ndofs()
    r = _cuda(W.random_vector(n, seed=800))
    R = _cuda(np.stack([W.random_vector(n, seed=810 + c) for c in range(3)]))
    other = _cuda(W.random_vector(n, seed=820))
    P.set_precision(fp32)
    try:
        P.set_graphs(False)
        z0 = P.vcycle(r).clone()
        Z0 = P.vcycle_multi(R).clone()
        P.set_graphs(True)
        for rep in range(4):
            y = P.apply(w.n_levels - 1, other)  # eager work between the replays
            torch.cuda.synchronize()
            z = P.vcycle(r)
            Z = P.vcycle_multi(R)
            torch.cuda.synchronize()
            assert torch.equal(z, z0), rep
            assert torch.equal(Z, Z0), rep
            assert torch.isfinite(y).all()
    finally:
        P.set_precision(False)


def test_solve_with_and_without_graphs(case):
    import torch

    w, P = case
    b = _cuda(P.rhs_manufactured())
    P.set_graphs(False)
    x0, i0 = P.solve(b, rtol=1e-8, maxit=300)
    x0 = x0.clone()
    P.set_graphs(True)
    for rep in range(2):
        x1, i1 = P.solve(b, rtol=1e-8, maxit=300)
        assert i1["iterations"] == i0["iterations"] and torch.equal(x1, x0), rep


def test_timing_counts_every_replay(case):
    w, P = case
    n = P.ndofs()
    r = _cuda(W.random_vector(n, seed=830))
    fine = w.n_levels - 1
    counts = {}
    for graphs in (False, True):
        P.set_graphs(graphs)
        P.timing(["cut_solve"], level=fine)
        for _ in range(3):
            P.vcycle(r)
        counts[graphs] = P.timing_read("cut_solve", fine)
        P.timing([])
    print(f"  timed cut launches: eager {counts[False]}, graph replays {counts[True]}")
    assert counts[True][0] == counts[False][0] > 0
    assert counts[True][1] > 0
    P.set_graphs(True)
