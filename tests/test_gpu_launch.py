"""The launch configurations of large levels, forced on small ones, against the
default configuration (bitwise) and against the CPU oracle, through the C ABI.

A full-size level runs its cut colour steps with one THREADS-wide block per
patch and its operator and interior-patch kernels with grid-stride loops over a
capped grid; the small parity cases would otherwise only run the twice-as-wide
cut-patch blocks and single-trip grids.  cmg_set_launch forces each choice.

Every case prints its name first so that a failing GPU run can be located."""
import numpy as np
import pytest

import oracle_cache
import workloads as W

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

CASES = [W.ball_q2().with_levels(3), W.offcentre_ball(3, 2), W.offcentre_disc(2, 4), W.ball_union(2, 3)]
# (small_cut_launch, max_blocks): THREADS-wide cut blocks; one or a few blocks
# per grid (every block makes many grid-stride trips); both together
POLICIES = [(0, 2048), (1536, 1), (1536, 3), (0, 2)]


@pytest.fixture(scope="module", params=CASES, ids=lambda w: w.name)
def case(request):
    import torch
    from paper_2508_11608_amd import Problem

    w = request.param
    print(f"\n[case] {w.name} dim={w.dim} k={w.k} levels={w.n_levels} (launch policies)", flush=True)
    P = Problem(w)
    levels, mats, prols, H = oracle_cache.build(w)
    yield w, P, levels, mats, H
    P.close()
    torch.cuda.synchronize()


def _cuda(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _results(w, P, levels, fp32):
    """Operator on every level, the first colour steps of both kinds, both
    smoothers and one V-cycle on the finest level, in one precision."""
    out = {}
    P.set_precision(fp32)
    try:
        for l in range(len(levels)):
            out[("apply", l)] = P.apply(l, _cuda(W.random_vector(levels[l].n_dofs, seed=300 + l))).cpu().numpy()
        L = len(levels) - 1
        n = levels[L].n_dofs
        b = _cuda(W.random_vector(n, seed=310))
        for interior in (True, False):
            for colour in range(2 ** w.dim):
                x = _cuda(W.random_vector(n, seed=320 + colour))
                P.colour_step(L, interior, colour, x, b)
                out[("colour", interior, colour)] = x.cpu().numpy()
        for post in (False, True):
            x = _cuda(W.random_vector(n, seed=330 + post))
            P.smooth(L, post, x, b)
            out[("smooth", post)] = x.cpu().numpy()
        out["vcycle"] = P.vcycle(_cuda(W.random_vector(n, seed=340))).cpu().numpy()
    finally:
        P.set_precision(False)
        P.set_launch()
    return out


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("policy", POLICIES, ids=lambda p: f"small{p[0]}-blocks{p[1]}")
def test_forced_launch_equals_default_bitwise(case, policy, fp32):
    w, P, levels, _, _ = case
    ref = _results(w, P, levels, fp32)
    P.set_launch(*policy)
    got = _results(w, P, levels, fp32)
    for key in ref:
        assert np.array_equal(got[key], ref[key]), key


@pytest.mark.parametrize("policy", POLICIES, ids=lambda p: f"small{p[0]}-blocks{p[1]}")
def test_forced_launch_matches_oracle(case, policy):
    """FP64 results of every forced configuration against the oracle."""
    w, P, levels, mats, H = case
    P.set_launch(*policy)
    got = _results(w, P, levels, False)
    for l in range(len(levels)):
        x = W.random_vector(levels[l].n_dofs, seed=300 + l)
        assert _rel(got[("apply", l)], mats[l] @ x) < 1e-12, l
    L = len(levels) - 1
    n = levels[L].n_dofs
    b = W.random_vector(n, seed=310)
    for post in (False, True):
        x = W.random_vector(n, seed=330 + post)
        H.smooth(L, x, b, post=post)
        assert _rel(got[("smooth", post)], x) < 1e-11, post
    assert _rel(got["vcycle"], H.vcycle(W.random_vector(n, seed=340))) < 1e-10
