"""Pins of the assembled CutFEM operator, ghost penalty and transfers."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import problem
from oracle.assemble import FormParams, ghost_face_matrix, uncut_cell_matrix
from oracle.basis import gll_nodes
from oracle.multigrid import build_patches, cartesian_patch_laplacian


def _sphere_data(w):
    c = np.array(w.centers[0])
    r = w.semi[0][0]
    d = w.dim
    gam = 2 * math.pi * r if d == 2 else 4 * math.pi * r * r
    vol = math.pi * r * r if d == 2 else 4 / 3 * math.pi * r ** 3
    return c, r, d, gam, vol


@pytest.fixture(scope="module", params=["disc2", "disc3", "ball2"])
def small(request):
    w = {"disc2": W.offcentre_disc(2, 3), "disc3": W.offcentre_disc(3, 3),
         "ball2": W.offcentre_ball(2, 2)}[request.param]
    levels, mats, prols, _ = problem.build(w, with_hierarchy=False)
    return w, levels, mats, prols


def test_nitsche_identities(small):
    """A(1,1) = gamma_D/h |Gamma|; A(1,x) = gamma_D/h int_Gamma x;
    A(x,x) = -|Omega| + gamma_D/h int_Gamma x^2; A(x^2,1) = -2|Omega| + gamma_D/h int_Gamma x^2
    (Nitsche form on polynomials; ghost terms vanish on global polynomials)."""
    w, levels, mats, _ = small
    lev, A = levels[-1], mats[-1]
    h, g = lev.h, w.gamma_D
    c, r, d, gam, vol = _sphere_data(w)
    X = lev.dof_coords()
    one = np.ones(lev.n_dofs)
    x1 = X[:, 0]
    int_x2 = c[0] ** 2 * gam + r * r * gam / d
    assert abs(one @ A @ one / (g / h * gam) - 1) < 1e-12
    assert abs(one @ A @ x1 / (g / h * c[0] * gam) - 1) < 1e-11
    assert abs(x1 @ A @ x1 / (-vol + g / h * int_x2) - 1) < 1e-12
    if w.k >= 2:
        assert abs(one @ A @ x1 ** 2 / (-2 * vol + g / h * int_x2) - 1) < 1e-12


def test_symmetric_positive_definite(small):
    _, levels, mats, _ = small
    for A in mats[:2]:
        Ad = A.toarray()
        assert np.abs(Ad - Ad.T).max() <= 1e-13 * np.abs(Ad).max()
        assert np.linalg.eigvalsh(Ad)[0] > 0


def test_ghost_face_kink_k1():
    """Q1, 2-D, two cells side by side in x, u = |x - x_F|: [d_x u] = -2 on the face,
    so u^T G u = gamma_g h^(2m-1) * 4 * h (m = 1)."""
    h, gam = 0.3, 0.1
    G = ghost_face_matrix(1, 2, h, 0, FormParams(gamma_D=40, gamma_g=gam))
    # local order x fastest: T1 nodes (x=-h,0) x (y=0,h), T2 nodes (0,h) x (0,h)
    u = np.array([h, 0, h, 0, 0, h, 0, h])
    assert abs(u @ G @ u - gam * h * 4 * h) < 1e-14
    # printed exponent 2m+1 scales by h^2
    G1 = ghost_face_matrix(1, 2, h, 0, FormParams(gamma_D=40, gamma_g=gam, ghost_exp_mode=1))
    assert abs(u @ G1 @ u - gam * h ** 3 * 4 * h) < 1e-14


def test_ghost_face_second_derivative_k2():
    """Q2, 2-D, u = (x - x_F)^2 on T2 only (zero on T1): first derivative continuous,
    [d_x^2 u] = 0 - 2 = -2, so u^T G u = gamma h^3/(2!)^2 * 4 * h."""
    h, gam = 0.25, 0.1
    G = ghost_face_matrix(2, 2, h, 0, FormParams(gamma_D=120, gamma_g=gam))
    xi = gll_nodes(2)
    t1 = np.zeros(9)
    t2 = np.array([(xi[i] * h) ** 2 for j in range(3) for i in range(3)])
    u = np.concatenate([t1, t2])
    assert abs(u @ G @ u - gam * h ** 3 / 4 * 4 * h) < 1e-14


def test_ghost_kernel_contains_polynomials():
    k, d, h = 3, 2, 0.2
    G = ghost_face_matrix(k, d, h, 1, FormParams(gamma_D=240, gamma_g=0.1))
    xi = gll_nodes(k)
    pts = []
    for cell_y in (0, 1):
        for j in range(k + 1):
            for i in range(k + 1):
                pts.append((xi[i] * h, (cell_y + xi[j]) * h))
    pts = np.array(pts)
    for p in [lambda x, y: x ** 3 * y, lambda x, y: y ** 3 - x * y ** 2, lambda x, y: x * x * y * y]:
        u = p(pts[:, 0], pts[:, 1])
        assert abs(u @ G @ u) < 1e-12


def test_prolongation_reproduces_coarse_polynomials(small):
    w, levels, _, prols = small
    k = w.k
    for l in range(1, len(levels)):
        Xc = levels[l - 1].dof_coords()
        Xf = levels[l].dof_coords()
        for p in range(k + 1):
            fc = Xc[:, 0] ** p * Xc[:, -1] ** (k - p)
            ff = Xf[:, 0] ** p * Xf[:, -1] ** (k - p)
            assert np.abs(prols[l - 1] @ fc - ff).max() < 1e-12


def test_interior_patch_matrix_is_principal_submatrix(small):
    w, levels, mats, _ = small
    lev, A = levels[-1], mats[-1]
    Ac = cartesian_patch_laplacian(w.k, w.dim, lev.h)
    groups = build_patches(lev, A)
    n_int = 0
    for (interior, _), ps in groups.items():
        if not interior:
            continue
        for dofs in ps.dofs:
            assert np.abs(A[dofs][:, dofs].toarray() - Ac).max() < 1e-12 * np.abs(Ac).max()
            n_int += 1
    assert n_int > 0 or w.dim == 3


def test_cartesian_patch_is_kronecker_sum():
    """Patch Laplacian = sum_i M x ... x K (i-th) x ... x M with 1-D patch matrices."""
    k, d, h = 2, 3, 0.125
    K1 = np.zeros((2 * k + 1,) * 2)
    M1 = np.zeros((2 * k + 1,) * 2)
    from oracle.basis import eval_basis, gauss_legendre
    x, wq = gauss_legendre(k + 1)
    B = eval_basis(k, x)
    D = eval_basis(k, x, 1)
    for c in (0, 1):
        sl = slice(k * c, k * c + k + 1)
        K1[sl, sl] += (D * wq[:, None]).T @ D / h
        M1[sl, sl] += (B * wq[:, None]).T @ B * h
    K1, M1 = K1[1:-1, 1:-1], M1[1:-1, 1:-1]
    ref = (np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1)) + np.kron(K1, np.kron(M1, M1)))
    assert np.abs(cartesian_patch_laplacian(k, d, h) - ref).max() < 1e-13


def test_ghost_orders_take_their_own_parameter():
    """Q2, 2-D, per-order parameters (gamma_1, gamma_2): a kink u = |x - x_F| only
    has a first-derivative jump and sees gamma_1 alone (u^T G u = gamma_1 h 4 h),
    the C^1 function (x - x_F)^2 on T2 only sees gamma_2 alone
    (u^T G u = gamma_2 h^3 / 4 * 4 h); gamma_g is then irrelevant."""
    h = 0.25
    fp = FormParams(gamma_D=120, gamma_g=0.5, gamma_m=(0.07, 0.13))
    G = ghost_face_matrix(2, 2, h, 0, fp)
    xi = gll_nodes(2)
    kink = np.concatenate([np.array([(1 - xi[i]) * h for j in range(3) for i in range(3)]),
                           np.array([xi[i] * h for j in range(3) for i in range(3)])])
    assert abs(kink @ G @ kink - 0.07 * h * 4 * h) < 1e-14
    c1 = np.concatenate([np.zeros(9), np.array([(xi[i] * h) ** 2 for j in range(3) for i in range(3)])])
    assert abs(c1 @ G @ c1 - 0.13 * h ** 3 / 4 * 4 * h) < 1e-14
