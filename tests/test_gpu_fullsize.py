"""The benchmark's workload at its full size, in the launch configuration the
benchmark times: the ball |x| < 0.7, Q2, 6 levels to 128^3 cells (3,246,717
DoFs), whose finest level runs THREADS-wide cut-patch blocks and capped
grid-stride grids with many trips per block.

The oracle cannot assemble or factorise the whole finest level quickly, so it
computes sampled outputs one by one from its own element matrices: rows of the
operator (uncut and cut cells, ghost faces) and the updates of sampled patches
of one cut and one interior colour step.  Nodes that a colour step must leave
alone are checked over the whole level, and the whole V-cycle and operator
are checked for symmetry.  Every case prints its name first so that a failing
GPU run can be located."""
import numpy as np
import pytest

import workloads as W
from oracle_rows import OracleRows

try:  # import at collection time: the first import on a fresh machine is slow
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

WL = W.ball_q2()


@pytest.fixture(scope="module")
def full():
    import torch
    from paper_2508_11608_amd import Problem

    print(f"\n[case] {WL.name} at full size ({WL.fine_cells}^3 cells)", flush=True)
    P = Problem(WL)
    R = OracleRows(WL)
    assert P.ndofs() == R.L.n_dofs
    yield P, R
    P.close()
    torch.cuda.synchronize()


def _cuda(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sample_dofs(R, rng, n_cut, n_any):
    """DoFs on cut cells (near the boundary, with Nitsche and ghost terms) and anywhere."""
    cuts = np.argwhere(R.L.cut)
    near = []
    for c in cuts[rng.choice(len(cuts), n_cut, replace=False)]:
        dofs = R.L.cell_dofs(tuple(int(v) for v in c))
        near.append(int(dofs[rng.integers(len(dofs))]))
    return near + [int(v) for v in rng.choice(R.L.n_dofs, n_any, replace=False)]


def test_operator_rows(full):
    P, R = full
    print("  [case] operator rows at full size", flush=True)
    L = WL.n_levels - 1
    x = W.random_vector(R.L.n_dofs, seed=1201)
    y = P.apply(L, _cuda(x)).cpu().numpy()
    rng = np.random.default_rng(1202)
    worst = 0.0
    for i in _sample_dofs(R, rng, 40, 24):
        cols, vals = R.row(i)
        ref = vals @ x[cols]
        err = abs(y[i] - ref) / np.abs(vals * x[cols]).sum()
        worst = max(worst, err)
    print(f"  64 sampled rows: max error {worst:.2e} (relative to sum |A_ij x_j|)")
    assert worst < 1e-12


def test_operator_symmetry(full):
    P, R = full
    print("  [case] operator symmetry at full size", flush=True)
    L = WL.n_levels - 1
    x = _cuda(W.random_vector(R.L.n_dofs, seed=1211))
    y = _cuda(W.random_vector(R.L.n_dofs, seed=1212))
    a = float(P.apply(L, x).dot(y))
    b = float(x.dot(P.apply(L, y)))
    print(f"  <Ax,y> = {a:.15e}, <x,Ay> = {b:.15e}")
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def _patch_update(R, V, x, b, interior):
    """x + A_j^{-1} (b - A x) on the internal DoFs of the patch at vertex V."""
    from oracle.multigrid import cartesian_patch_laplacian

    I = R.patch_internal(V)
    rows = [R.row(int(i)) for i in I]
    r = np.array([b[i] - vals @ x[cols] for i, (cols, vals) in zip(I, rows)])
    if interior:
        Aj = cartesian_patch_laplacian(R.k, R.d, R.L.h)
    else:
        pos = {int(j): n for n, j in enumerate(I)}
        Aj = np.zeros((len(I), len(I)))
        for a, (cols, vals) in enumerate(rows):
            for c, v in zip(cols, vals):
                if int(c) in pos:
                    Aj[a, pos[int(c)]] += v
    return I, x[I] + np.linalg.solve(Aj, r)


@pytest.mark.parametrize("interior,colour", [(False, 0), (False, 5), (True, 3)], ids=["cut-c0", "cut-c5", "interior-c3"])
def test_colour_step_sampled_patches(full, interior, colour):
    P, R = full
    print(f"  [case] {'interior' if interior else 'cut'} colour step {colour} at full size", flush=True)
    L = WL.n_levels - 1
    n = R.L.n_dofs
    x = W.random_vector(n, seed=1220 + colour)
    b = W.random_vector(n, seed=1230 + colour)
    xg = _cuda(x)
    P.colour_step(L, interior, colour, xg, _cuda(b))
    xn = xg.cpu().numpy()
    cut_v, int_v = R.patch_masks(colour)
    vmask = int_v if interior else cut_v
    verts = np.argwhere(vmask)
    print(f"  {len(verts)} patches in the colour", flush=True)
    # nodes outside the colour's patches are left exactly as they were
    inside = R.internal_node_mask(vmask)
    node_dof = R.L.dof_of_node[inside]
    touched = np.zeros(n, dtype=bool)
    touched[node_dof[node_dof >= 0]] = True
    assert np.array_equal(xn[~touched], x[~touched])
    # sampled patches against the oracle's local solves
    rng = np.random.default_rng(1240 + colour)
    worst = 0.0
    for v in verts[rng.choice(len(verts), 8, replace=False)]:
        I, ref = _patch_update(R, tuple(int(t) for t in v), x, b, interior)
        err = np.abs(xn[I] - ref).max() / max(np.abs(ref - x[I]).max(), 1e-300)
        worst = max(worst, err)
    print(f"  8 sampled patches: max error {worst:.2e} (relative to the patch correction)")
    assert worst < 1e-10


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_vcycle_symmetric_positive(full, fp32):
    P, R = full
    print(f"  [case] V-cycle symmetry at full size, fp32={fp32}", flush=True)
    n = R.L.n_dofs
    r1 = _cuda(W.random_vector(n, seed=1251))
    r2 = _cuda(W.random_vector(n, seed=1252))
    P.set_precision(fp32)
    try:
        z1 = P.vcycle(r1)
        z2 = P.vcycle(r2)
    finally:
        P.set_precision(False)
    a, b = float(z1.dot(r2)), float(r1.dot(z2))
    q = float(z1.dot(r1))
    print(f"  <Br1,r2> = {a:.15e}, <r1,Br2> = {b:.15e}, <Br1,r1> = {q:.6e}")
    assert q > 0.0
    assert abs(a - b) <= (1e-5 if fp32 else 1e-11) * q
