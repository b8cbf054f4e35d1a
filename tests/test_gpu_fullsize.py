"""The benchmark's workloads at their full size, in the launch configuration
the benchmark times: the ball |x| < 0.7, Q2, 6 levels to 128^3 cells (3,246,717
DoFs) and the union of 8 spheres, Q3, 5 levels to 64^3 cells (925,877 DoFs),
whose finest levels run THREADS-wide cut-patch blocks and capped grid-stride
grids with many trips per block; on the union also the 8-column V-cycle (FP64
all columns per patch block, FP32 local solves on the matrix cores).

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

WLS = [W.ball_q2(), W.sphere_union_8()]


@pytest.fixture(scope="module")
def built():
    """One library problem and one row oracle per workload, built on first use."""
    import torch

    cache = {}
    yield cache
    for P, _ in cache.values():
        P.close()
    torch.cuda.synchronize()


def _get(built, w):
    from paper_2508_11608_amd import Problem

    if w.name not in built:
        print(f"\n[case] {w.name} at full size ({w.fine_cells}^{w.dim} cells)", flush=True)
        P = Problem(w)
        R = OracleRows(w)
        assert P.ndofs() == R.L.n_dofs
        built[w.name] = (P, R)
    return built[w.name]


@pytest.fixture(scope="module", params=WLS, ids=lambda w: w.name)
def full(request, built):
    return (request.param,) + _get(built, request.param)


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
    w, P, R = full
    print(f"  [case] {w.name} operator rows at full size", flush=True)
    L = w.n_levels - 1
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
    w, P, R = full
    print(f"  [case] {w.name} operator symmetry at full size", flush=True)
    L = w.n_levels - 1
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
    return I, x[I] + np.linalg.solve(Aj, r), np.linalg.cond(Aj)


@pytest.mark.parametrize("interior,colour,fp32", [(False, 0, False), (False, 5, False), (True, 3, False),
                                                (False, 0, True), (True, 3, True)],
                         ids=["cut-c0", "cut-c5", "interior-c3", "cut-c0-fp32", "interior-c3-fp32"])
def test_colour_step_sampled_patches(full, interior, colour, fp32):
    w, P, R = full
    print(f"  [case] {w.name} {'interior' if interior else 'cut'} colour step {colour} at full size, fp32={fp32}",
          flush=True)
    L = w.n_levels - 1
    n = R.L.n_dofs
    x = W.random_vector(n, seed=1220 + colour)
    b = W.random_vector(n, seed=1230 + colour)
    xg = _cuda(x)
    P.set_precision(fp32)
    try:
        P.colour_step(L, interior, colour, xg, _cuda(b))
    finally:
        P.set_precision(False)
    xn = xg.cpu().numpy()
    cut_v, int_v = R.patch_masks(colour)
    vmask = int_v if interior else cut_v
    verts = np.argwhere(vmask)
    print(f"  {len(verts)} patches in the colour", flush=True)
    # nodes outside the colour's patches are left exactly as they were (in FP32
    # the step runs on x rounded to FP32)
    inside = R.internal_node_mask(vmask)
    node_dof = R.L.dof_of_node[inside]
    touched = np.zeros(n, dtype=bool)
    touched[node_dof[node_dof >= 0]] = True
    x_in = x.astype(np.float32).astype(np.float64) if fp32 else x
    assert np.array_equal(xn[~touched], x_in[~touched])
    # sampled patches against the oracle's local solves
    rng = np.random.default_rng(1240 + colour)
    worst, worst_cond = 0.0, 0.0
    for v in verts[rng.choice(len(verts), 8, replace=False)]:
        I, ref, cond = _patch_update(R, tuple(int(t) for t in v), x, b, interior)
        # FP64: relative to the patch correction; FP32: to the updated values
        # (the FP32 step also rounds x itself)
        scale = np.abs(ref).max() if fp32 else np.abs(ref - x[I]).max()
        err = np.abs(xn[I] - ref).max() / max(scale, 1e-300)
        print(f"    patch {tuple(int(t) for t in v)}: {len(I)} DoFs, cond {cond:.1e}, error {err:.2e}")
        # both sides solve the same local system, the library in FP64 or with
        # the FP32 rounding of the FP64 inverse and FP32 arithmetic: the
        # difference is bounded by the condition number times the rounding unit
        assert err < (1e-5 + 1e-6 * cond if fp32 else 1e-10 + 1e-14 * cond)
        worst, worst_cond = max(worst, err), max(worst_cond, cond)
    print(f"  8 sampled patches: max error {worst:.2e}, max cond {worst_cond:.1e}")


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_vcycle_symmetric_positive(full, fp32):
    w, P, R = full
    print(f"  [case] {w.name} V-cycle symmetry at full size, fp32={fp32}", flush=True)
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


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_union8_eight_column_vcycle(built, fp32):
    """The 8-column V-cycle of the Q3 union (FP64: every inverse and cell row
    read once for all columns; FP32: local solves on the matrix cores): each
    column against the one-column V-cycle of the same precision and against
    the FP64 one, and the 8 x 8 matrix <B r_a, r_b> symmetric."""
    import torch

    w = WLS[1]
    P, R = _get(built, w)
    print(f"  [case] {w.name} 8-column V-cycle at full size, fp32={fp32}", flush=True)
    n = R.L.n_dofs
    Rm = _cuda(W.random_vector(n, seed=1261, nrhs=8))
    z64 = torch.stack([P.vcycle(Rm[c].contiguous()) for c in range(8)])
    P.set_precision(fp32)
    try:
        Z = P.vcycle_multi(Rm)
        single = torch.stack([P.vcycle(Rm[c].contiguous()) for c in range(8)])
    finally:
        P.set_precision(False)
    scale = float(z64.abs().max())
    d_multi = float((Z - z64).abs().max()) / scale
    d_single = float((single - z64).abs().max()) / scale
    M = (Z @ Rm.T).cpu().numpy()
    asym = np.abs(M - M.T).max() / np.abs(np.diag(M)).max()
    print(f"  vs FP64 one-column V-cycles: 8-column {d_multi:.2e}, one-column {d_single:.2e}; asymmetry {asym:.2e}")
    if fp32:
        assert d_multi <= 10.0 * d_single + 1e-6
        assert asym < 1e-5
    else:
        assert d_multi < 1e-11
        assert asym < 1e-11
    assert np.all(np.diag(M) > 0.0)
