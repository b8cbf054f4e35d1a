"""Pins of the patch smoother, V-cycle and PCG of the oracle."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spl

import workloads as W
from oracle import problem
from oracle.assemble import l2_error
from oracle.multigrid import Hierarchy, gmres, pcg, vcycle_iteration


def _hier(w, L=None, gamma_g=None):
    if gamma_g is not None:
        w = W.Workload(**{**w.__dict__, "gamma_g": gamma_g})
        levels, mats, prols, _ = problem.build(w, n_levels=L, with_hierarchy=False)
        # without ghost penalty small cuts can make local matrices indefinite;
        # the identity tested with it is purely algebraic
        return w, levels, mats, prols, Hierarchy(levels, mats, prols, n_c=w.n_c, require_spd=False)
    levels, mats, prols, H = problem.build(w, n_levels=L)
    return w, levels, mats, prols, H


@pytest.fixture(scope="module")
def disc3():
    return _hier(W.offcentre_disc(2, 3))


def test_patches_disjoint_within_colour_and_cover(disc3):
    _, levels, _, _, H = disc3
    for l in range(1, len(levels)):
        seen = np.zeros(levels[l].n_dofs, dtype=int)
        for ps in H.patches[l].values():
            allc = np.concatenate(ps.dofs)
            assert len(np.unique(allc)) == len(allc)  # disjoint within a colour class
            seen[allc] += 1
        assert seen.min() >= 1  # every DoF is smoothed


def _colour_operator(H, l, key, n):
    """B_c = sum_j Q_j^T A_j^{-1} Q_j with A_j^{-1} the stored local inverse."""
    Bc = np.zeros((n, n))
    ps = H.patches[l].get(key)
    if ps is None:
        return Bc
    for dofs, inv in zip(ps.dofs, ps.invs):
        Bc[np.ix_(dofs, dofs)] += inv
    return Bc


def _same_colour_coupling(A, ps):
    worst = 0.0
    for i, d1 in enumerate(ps.dofs):
        for d2 in ps.dofs[i + 1:]:
            worst = max(worst, np.abs(A[np.ix_(d1, d2)]).max())
    return worst


def test_sequential_mvs_without_ghost_equals_coloured():
    """With gamma_g = 0 same-coloured patches do not couple (A[I_j, I_j'] = 0), so
    the simultaneous update of a colour equals the sequential MVS over its patches:
    every correction solves its own local problem with the residual at the start
    of the step.  Checked as a backward error because local matrices without
    ghost penalty have condition numbers up to ~1e7."""
    w, levels, mats, _, H = _hier(W.offcentre_disc(2, 3), gamma_g=0.0)
    l = len(levels) - 1
    A = mats[l].toarray()
    n = A.shape[0]
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    r0 = b - A @ x0
    for key in H.schedule(l):
        ps = H.patches[l].get(key)
        if ps is None:
            continue
        assert _same_colour_coupling(A, ps) == 0.0
        x = x0.copy()
        H.colour_step(l, key, x, b)
        dx = x - x0
        touched = np.zeros(n, dtype=bool)
        for dofs in ps.dofs:
            Aj = A[np.ix_(dofs, dofs)]
            res = Aj @ dx[dofs] - r0[dofs]
            assert np.abs(res).max() <= 1e-8 * (np.abs(Aj).max() * np.abs(dx[dofs]).max() + np.abs(r0[dofs]).max())
            touched[dofs] = True
        assert np.all(dx[~touched] == 0.0)


def test_ghost_penalty_couples_same_coloured_cut_patches(disc3):
    """The inconsistency of the parallel smoother: with gamma_g > 0 some
    same-coloured cut patches couple through ghost faces."""
    _, levels, mats, _, H = disc3
    l = len(levels) - 1
    A = mats[l].toarray()
    worst = max(_same_colour_coupling(A, ps) for (interior, _), ps in H.patches[l].items() if not interior)
    assert worst > 0.0


def test_two_grid_formula(disc3):
    """Two-level V-cycle == (I - E_post (I - P A0^{-1} P^T A) E_pre) A^{-1}, with
    E = prod_c (I - B_c A) over the colour schedule."""
    w, levels, mats, prols, _ = disc3
    H = Hierarchy(levels[:2], mats[:2], prols[:1], n_c=w.n_c)
    A = mats[1].toarray()
    n = A.shape[0]
    I = np.eye(n)
    E_pre = I.copy()
    for key in H.schedule(1):
        E_pre = (I - _colour_operator(H, 1, key, n) @ A) @ E_pre
    E_post = I.copy()
    for key in H.schedule(1, post=True):
        E_post = (I - _colour_operator(H, 1, key, n) @ A) @ E_post
    P = prols[0].toarray()
    A0 = mats[0].toarray()
    E = E_post @ (I - P @ np.linalg.solve(A0, P.T @ A)) @ E_pre
    B_ref = (I - E) @ np.linalg.inv(A)
    B = np.column_stack([H.vcycle(e) for e in I])
    assert np.abs(B - B_ref).max() < 1e-10 * np.abs(B_ref).max()


def test_vcycle_symmetric_positive(disc3):
    _, levels, mats, _, H = disc3
    n = levels[-1].n_dofs
    B = np.column_stack([H.vcycle(e) for e in np.eye(n)])
    assert np.abs(B - B.T).max() < 1e-12 * np.abs(B).max()
    ev = np.linalg.eigvals(B @ mats[-1].toarray()).real
    # exact patch solvers would bound the spectrum by 1; the ignored ghost
    # coupling between same-coloured patches lets it exceed 1 by a little
    assert ev.min() > 0.1 and ev.max() < 1.01


def test_vcycle_q3_spd():
    w, levels, mats, _, H = _hier(W.offcentre_disc(3, 3))
    n = levels[-1].n_dofs
    B = np.column_stack([H.vcycle(e) for e in np.eye(n)])
    assert np.abs(B - B.T).max() < 1e-11 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0


def test_pcg_matches_direct_solve():
    w, levels, mats, _, H = _hier(W.disc_q2())
    b = problem.rhs(w, levels[-1])
    x, it, hist = pcg(mats[-1], b, H.vcycle, rtol=1e-12)
    xs = spl.spsolve(mats[-1].tocsc(), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9
    assert it <= 12


@pytest.mark.parametrize("k", [1, 2])
def test_l2_convergence_rate(k):
    w = W.disc_q2().with_degree(k)
    u, _, _ = problem.manufactured(2)
    errs = []
    for L in (4, 5):
        levels, mats, _, H = problem.build(w, n_levels=L)
        b = problem.rhs(w, levels[-1])
        x, _, _ = pcg(mats[-1], b, H.vcycle, rtol=1e-11)
        errs.append(l2_error(levels[-1], problem.shapes_of(w), problem.form_params(w), x, u))
    assert math.log2(errs[0] / errs[1]) >= k + 0.8


def _discrete_l2_errors(w, Ls):
    """L2 errors of the discrete solutions of the manufactured problem on the
    finest levels Ls, each solved by Jacobi-scaled CG to 1e-12 (the solution
    of A x = b, independent of the multigrid under test elsewhere)."""
    import scipy.sparse as sp

    from oracle.assemble import assemble
    from oracle.geometry import build_levels

    u, _, _ = problem.manufactured(w.dim)
    shapes, fp = problem.shapes_of(w), problem.form_params(w)
    errs = []
    for L in Ls:
        lev = build_levels(shapes, w.dim, w.k, L, w.coarse_cells, w.lo, w.hi)[-1]
        A = assemble(lev, shapes, fp)
        b = problem.rhs(w, lev)
        d = 1.0 / np.sqrt(A.diagonal())
        D = sp.diags(d)
        y, info = spl.cg(D @ A @ D, d * b, rtol=1e-12, maxiter=20000)
        assert info == 0
        errs.append(l2_error(lev, shapes, fp, d * y, u))
    return errs


@pytest.mark.parametrize("k", [1, 2])
def test_l2_convergence_rate_ball(k):
    """O(h^(k+1)) in 3-D: the ball |x| < 0.7 at 16^3 and 32^3 cells."""
    errs = _discrete_l2_errors(W.ball_q2().with_degree(k), (3, 4))
    assert math.log2(errs[0] / errs[1]) >= k + 0.8, errs


def test_l2_convergence_rate_disc_q3():
    """O(h^4) for Q3 on the disc at 32^2 and 64^2 cells."""
    errs = _discrete_l2_errors(W.disc_q2().with_degree(3), (4, 5))
    assert math.log2(errs[0] / errs[1]) >= 3 + 0.8, errs


# ---- outer solvers of the paper's tables: GMRES and the V-cycle iteration ----

def test_gmres_matches_an_independent_implementation():
    """The oracle's right-preconditioned restarted GMRES against SciPy's GMRES
    (an independent implementation) on a non-symmetric system: the same number
    of inner iterations and the same residual to a few digits."""
    import scipy.sparse as sp

    rng = np.random.default_rng(0)
    n = 60
    A = sp.csr_matrix(4.0 * np.eye(n) + 0.3 * rng.standard_normal((n, n)))
    b = rng.standard_normal(n)
    x, it, hist = gmres(A, b, lambda v: v, rtol=1e-10, restart=10, maxit=200)
    count = [0]

    def cb(_):
        count[0] += 1

    xs, info = spl.gmres(A, b, rtol=1e-10, restart=10, maxiter=200, callback=cb, callback_type="pr_norm")
    assert info == 0 and it == count[0]
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel <= 1e-10 and abs(rel / (np.linalg.norm(b - A @ xs) / np.linalg.norm(b)) - 1) < 1e-3
    assert all(h1 >= h2 - 1e-15 for h1, h2 in zip(hist, hist[1:]))  # the GMRES residual never grows


def test_gmres_with_exact_preconditioner_takes_one_step(disc3):
    w, levels, mats, _, _ = disc3
    A = mats[-1].tocsc()
    b = problem.rhs(w, levels[-1])
    lu = spl.splu(A)
    x, it, _ = gmres(A, b, lu.solve, rtol=1e-12)
    assert it == 1
    assert np.abs(x - lu.solve(b)).max() <= 1e-10 * np.abs(x).max()


def test_gmres_vcycle_solves_the_cutfem_system(disc3):
    w, levels, mats, _, H = disc3
    A = mats[-1]
    b = problem.rhs(w, levels[-1])
    x, it, _ = gmres(A, b, H.vcycle, rtol=1e-9)
    xd = spl.spsolve(A.tocsc(), b)
    assert 1 <= it <= 30
    assert np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b) * 1.0000001
    assert np.abs(x - xd).max() <= 1e-6 * np.abs(xd).max()


def test_vcycle_iteration_closed_form():
    """x_k of the stand-alone V-cycle is sum_{i<k} (I - B A)^i B b: the V-cycle
    is a linear map, so its dense matrix B (columns B e_j) gives the closed form."""
    w, levels, mats, prols, H = _hier(W.disc_q2(), L=2)
    A = mats[-1].toarray()
    n = A.shape[0]
    B = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    b = problem.rhs(w, levels[-1])
    M = np.eye(n) - B @ A
    xk = np.zeros(n)
    term = B @ b
    for _ in range(3):
        xk += term
        term = M @ term
    x3, it, _ = vcycle_iteration(mats[-1], b, H.vcycle, rtol=0.0, maxit=3)
    assert it == 3
    assert np.abs(x3 - xk).max() <= 1e-12 * np.abs(xk).max()


# ---- patch-local residuals (ghost coupling beyond the patch closure dropped) ----

def _ghost_local(H):
    import copy

    Hl = copy.copy(H)  # shares matrices and patches
    Hl.ghost_local = True
    return Hl


def test_patch_local_residual_is_the_residual_of_x_masked_to_the_closure(disc3):
    """Brute force by coordinates: for every cut patch of a colour, the residual
    of the variant is (b - A x~)[I_j] with x~ = x on the DoFs whose coordinates
    lie in the closed box [X - h, X + h]^d and zero elsewhere."""
    _, levels, mats, _, H = disc3
    Hl = _ghost_local(H)
    l = len(levels) - 1
    lev = levels[l]
    X = lev.dof_coords()
    A = mats[l].toarray()
    n = lev.n_dofs
    rng = np.random.default_rng(5)
    x0, b = rng.standard_normal(n), rng.standard_normal(n)
    for key, ps in H.patches[l].items():
        if key[0]:
            continue
        want = x0.copy()
        for V, dofs, inv in zip(ps.vertices, ps.dofs, ps.invs):
            centre = lev.lo + np.asarray(V, dtype=np.float64) * lev.h
            inside = np.all(np.abs(X - centre) <= lev.h * (1 + 1e-12), axis=1)
            xt = np.where(inside, x0, 0.0)
            want[dofs] += inv @ (b - A @ xt)[dofs]
        got = x0.copy()
        Hl.colour_step(l, key, got, b)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), key


def test_patch_local_residual_without_ghost_penalty_is_exact():
    """With gamma_g = 0 there is no coupling beyond a patch closure: both
    variants give the same smoother."""
    w, levels, mats, _, H = _hier(W.offcentre_disc(2, 3), gamma_g=0.0)
    Hl = _ghost_local(H)
    l = len(levels) - 1
    rng = np.random.default_rng(6)
    b = rng.standard_normal(levels[l].n_dofs)
    x1, x2 = np.zeros_like(b), np.zeros_like(b)
    H.smooth(l, x1, b)
    Hl.smooth(l, x2, b)
    assert np.abs(x1 - x2).max() <= 1e-13 * np.abs(x1).max()


def test_patch_local_smoother_is_inconsistent(disc3):
    """The exact residual keeps the discrete solution fixed; the patch-local one
    moves it (the measured inconsistency), and its V-cycle is not symmetric."""
    w, levels, mats, _, H = disc3
    Hl = _ghost_local(H)
    l = len(levels) - 1
    b = problem.rhs(w, levels[l])
    xs = spl.spsolve(mats[l].tocsc(), b)
    x1, x2 = xs.copy(), xs.copy()
    H.smooth(l, x1, b)
    Hl.smooth(l, x2, b)
    assert np.linalg.norm(x1 - xs) <= 1e-11 * np.linalg.norm(xs)
    assert np.linalg.norm(x2 - xs) >= 1e-6 * np.linalg.norm(xs)
    n = levels[l].n_dofs
    B = np.column_stack([Hl.vcycle(e) for e in np.eye(n)])
    assert np.abs(B - B.T).max() > 1e-6 * np.abs(B).max()
    # as a preconditioner it still works: GMRES converges to the discrete solution
    x, it, _ = gmres(mats[l], b, Hl.vcycle, rtol=1e-10)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs) and it <= 30
