"""Assembled CutFEM operator A_l and load vector b_l (oracle; test infrastructure only).

Bilinear form (paper, Section 2.1, eq. (cutfem_nitsche) plus eq. (cutfem-ghost)):

  A(u, v) = (grad u, grad v)_Omega - (d_n u, v)_Gamma - (u, d_n v)_Gamma
            + (gamma_D / h)(u, v)_Gamma + g(u, v),

  g(u, v) = sum_{F in F_G} sum_{m=1..k} gamma_m h^{e(m)} / (m!)^2 ([d_n^m u], [d_n^m v])_F,

with F_G the faces between two active cells of which at least one is cut.
Readings (the paper prints the ghost scaling as h_F^{2k+1} with the sum from 0):
  * e(m) = 2m - 1 (stiffness scaling, mode 0) or 2m + 1 (as printed, mode 1);
  * the m = 0 jump of a continuous function vanishes and is dropped;
  * gamma_m = gamma_g for all m unless given per order (the paper tunes
    gamma_1, gamma_2, gamma_3 one by one, Section 4); h = h_F = h_l is the
    cell side length.
Load vector (paper eq. (weak-equation) plus the symmetric Nitsche terms for
non-zero Dirichlet data g):  b_i = (f, phi_i)_Omega + (g, (gamma_D/h) phi_i - d_n phi_i)_Gamma.

Every matrix is built entry by entry from quadrature of basis functions; the
uncut cell matrix uses a tensor Gauss rule with k+1 points (exact for Q_k
products), cut cells use the rule of oracle.quadrature.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .basis import eval_basis, eval_tensor_basis, gauss_legendre, local_index_tuples
from .geometry import Level
from .quadrature import cut_cell_rule_union


@dataclass
class FormParams:
    gamma_D: float          # Nitsche penalty; the penalty term is gamma_D / h
    gamma_g: float = 0.1    # ghost penalty, the same for every derivative order
    ghost_exp_mode: int = 0  # 0: h^(2m-1); 1: h^(2m+1)
    quad_n: int = 14        # Gauss points per smooth piece of a cut-cell rule
    quad_beta: float = 0.35  # subdivision threshold of the cut-cell rule
    union_depth: int = 4     # bisection depth of cells crossed by several surfaces
    gamma_m: tuple = ()      # per derivative order m = 1..; overrides gamma_g where given and > 0

    def gamma(self, m: int) -> float:
        return self.gamma_m[m - 1] if len(self.gamma_m) >= m and self.gamma_m[m - 1] > 0 else self.gamma_g


def tensor_gauss_ref(d: int, n: int):
    x, w = gauss_legendre(n)
    grid = np.stack(np.meshgrid(*[x] * d, indexing="ij"), axis=-1).reshape(-1, d)
    wgt = np.ones(1)
    for _ in range(d):
        wgt = np.multiply.outer(wgt, w)
    return grid, wgt.reshape(-1)


def uncut_cell_matrix(k: int, d: int, h: float) -> np.ndarray:
    """(grad phi_a, grad phi_b) over a whole cell of side h."""
    xi, w = tensor_gauss_ref(d, k + 1)
    E = np.zeros(((k + 1) ** d,) * 2)
    for i in range(d):
        G = eval_tensor_basis(k, xi, deriv_dirs=i) / h
        E += (G * w[:, None]).T @ G * h ** d
    return E


def cut_cell_matrix(level: Level, shapes, cell, fp: FormParams) -> np.ndarray:
    """Volume, Nitsche and penalty terms of one cut cell (shapes: list, Omega is their union)."""
    k, d, h = level.k, level.dim, level.h
    lo = level.cell_lo(cell)
    vx, vw, sx, sw, sn = cut_cell_rule_union(shapes, lo, lo + h, n=fp.quad_n, n_t=k + 1, beta=fp.quad_beta,
                                             union_depth=fp.union_depth)
    n_loc = (k + 1) ** d
    E = np.zeros((n_loc, n_loc))
    xi_v = (vx - lo) / h
    for i in range(d):
        G = eval_tensor_basis(k, xi_v, deriv_dirs=i) / h
        E += (G * vw[:, None]).T @ G
    if len(sw):
        xi_s = (sx - lo) / h
        V = eval_tensor_basis(k, xi_s)
        Dn = np.zeros_like(V)
        for i in range(d):
            Dn += sn[:, i : i + 1] * eval_tensor_basis(k, xi_s, deriv_dirs=i) / h
        VW = V * sw[:, None]
        E -= VW.T @ Dn + Dn.T @ VW
        E += (fp.gamma_D / h) * (VW.T @ V)
    return E


def ghost_face_matrix(k: int, d: int, h: float, direction: int, fp: FormParams) -> np.ndarray:
    """Ghost penalty of one face normal to `direction` between a lower cell T1
    and an upper cell T2, acting on [dofs(T1); dofs(T2)] (2 (k+1)^d unknowns).
    The jump is taken as (trace from T1 at its upper face) - (trace from T2 at
    its lower face)."""
    n_loc = (k + 1) ** d
    tang = [i for i in range(d) if i != direction]
    xf, wf = tensor_gauss_ref(d - 1, k + 1)
    P = len(wf)
    tup = local_index_tuples(k, d)
    G = np.zeros((2 * n_loc, 2 * n_loc))
    for m in range(1, k + 1):
        expo = 2 * m - 1 if fp.ghost_exp_mode == 0 else 2 * m + 1
        coef = fp.gamma(m) * h ** expo / math.factorial(m) ** 2
        J = np.zeros((P, 2 * n_loc))
        for side, xn in ((0, 1.0), (1, 0.0)):
            vals = np.ones((P, n_loc))
            for i in range(d):
                if i == direction:
                    b = eval_basis(k, np.array([xn]), m)[0] / h ** m  # (k+1,)
                    vals *= b[tup[:, i]][None, :]
                else:
                    t = xf[:, tang.index(i)] if d > 1 else np.zeros(P)
                    vals *= eval_basis(k, t, 0)[:, tup[:, i]]
            J[:, side * n_loc : (side + 1) * n_loc] = vals if side == 0 else -vals
        face_w = wf * h ** (d - 1)
        G += coef * (J * face_w[:, None]).T @ J
    return G


def ghost_faces(level: Level):
    """All faces of F_G as (direction, lower cell, upper cell)."""
    out = []
    N, d = level.N, level.dim
    for cell in level.active_cells():
        for i in range(d):
            if cell[i] + 1 >= N:
                continue
            nb = list(cell)
            nb[i] += 1
            nb = tuple(nb)
            if level.active[nb] and (level.cut[cell] or level.cut[nb]):
                out.append((i, cell, nb))
    return out


def assemble(level: Level, shapes, fp: FormParams, with_ghost: bool = True) -> sp.csr_matrix:
    """Global A_l in canonical DoF order."""
    k, d, h = level.k, level.dim, level.h
    n_loc = (k + 1) ** d
    rows, cols, vals = [], [], []
    K = uncut_cell_matrix(k, d, h)
    uncut = [c for c in level.active_cells() if not level.cut[c]]
    if uncut:
        D = np.stack([level.cell_dofs(c) for c in uncut])
        rows.append(np.repeat(D, n_loc, axis=1).reshape(-1))
        cols.append(np.tile(D, (1, n_loc)).reshape(-1))
        vals.append(np.tile(K.reshape(-1), len(uncut)))
    for c in level.active_cells():
        if level.cut[c]:
            E = cut_cell_matrix(level, shapes, c, fp)
            D = level.cell_dofs(c)
            rows.append(np.repeat(D, n_loc))
            cols.append(np.tile(D, n_loc))
            vals.append(E.reshape(-1))
    if with_ghost:
        Gd = [ghost_face_matrix(k, d, h, i, fp) for i in range(d)]
        for i, c1, c2 in ghost_faces(level):
            D = np.concatenate([level.cell_dofs(c1), level.cell_dofs(c2)])
            rows.append(np.repeat(D, 2 * n_loc))
            cols.append(np.tile(D, 2 * n_loc))
            vals.append(Gd[i].reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(level.n_dofs, level.n_dofs)).tocsr()
    A.sum_duplicates()
    return A


def load_vector(level: Level, shapes, fp: FormParams, f, g=None) -> np.ndarray:
    """b_i = (f, phi_i)_Omega + (g, (gamma_D/h) phi_i - d_n phi_i)_Gamma.

    f, g: callables on points of shape (P, d).  Uncut cells use a tensor Gauss
    rule with k+3 points per direction, cut cells the cut rule with n points per
    smooth piece in every direction."""
    k, d, h = level.k, level.dim, level.h
    b = np.zeros(level.n_dofs)
    xi_u, w_u = tensor_gauss_ref(d, k + 3)
    V_u = eval_tensor_basis(k, xi_u)
    for c in level.active_cells():
        lo = level.cell_lo(c)
        D = level.cell_dofs(c)
        if not level.cut[c]:
            x = lo + h * xi_u
            np.add.at(b, D, V_u.T @ (w_u * h ** d * f(x)))
            continue
        vx, vw, sx, sw, sn = cut_cell_rule_union(shapes, lo, lo + h, n=fp.quad_n, n_t=fp.quad_n,
                                                 beta=fp.quad_beta, union_depth=fp.union_depth)
        loc = eval_tensor_basis(k, (vx - lo) / h).T @ (vw * f(vx))
        if g is not None and len(sw):
            xi_s = (sx - lo) / h
            V = eval_tensor_basis(k, xi_s)
            Dn = np.zeros_like(V)
            for i in range(d):
                Dn += sn[:, i : i + 1] * eval_tensor_basis(k, xi_s, deriv_dirs=i) / h
            gw = g(sx) * sw
            loc += (fp.gamma_D / h) * (V.T @ gw) - Dn.T @ gw
        np.add.at(b, D, loc)
    return b


def l2_error(level: Level, shapes, fp: FormParams, x: np.ndarray, u_exact) -> float:
    """|| u_h - u ||_{L2(Omega)} using the same rules as the load vector."""
    k, d, h = level.k, level.dim, level.h
    xi_u, w_u = tensor_gauss_ref(d, k + 3)
    V_u = eval_tensor_basis(k, xi_u)
    acc = 0.0
    for c in level.active_cells():
        lo = level.cell_lo(c)
        xc = x[level.cell_dofs(c)]
        if not level.cut[c]:
            pts = lo + h * xi_u
            acc += np.sum(w_u * h ** d * (V_u @ xc - u_exact(pts)) ** 2)
            continue
        vx, vw, *_ = cut_cell_rule_union(shapes, lo, lo + h, n=fp.quad_n, n_t=fp.quad_n, beta=fp.quad_beta,
                                         union_depth=fp.union_depth)
        acc += np.sum(vw * (eval_tensor_basis(k, (vx - lo) / h) @ xc - u_exact(vx)) ** 2)
    return math.sqrt(acc)
