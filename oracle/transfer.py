"""Intergrid operators (oracle; test infrastructure only).

Prolongation = embedding V_{l-1} -> V_l (paper, Section 2.2): the fine
coefficient of DoF i is the coarse finite element function evaluated at the
fine node x_i, which is well defined because Omega_l is contained in
Omega_{l-1}.  Restriction is the transpose (Euclidean inner product on
coefficient vectors, end of Section 2.2).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .basis import eval_tensor_basis
from .geometry import Level


def _coarse_cells_containing(fine: Level, node: tuple):
    """Coarse cells whose closure contains the fine lattice node."""
    k = fine.k
    per_dim = []
    for I in node:
        if I % k == 0:
            v = I // k  # fine vertex index
            if v % 2 == 0:
                cands = [v // 2 - 1, v // 2]
            else:
                cands = [(v - 1) // 2]
        else:
            cands = [(I // k) // 2]
        per_dim.append([c for c in cands if 0 <= c < fine.N // 2])
    return list(itertools.product(*per_dim))


def prolongation(coarse: Level, fine: Level) -> sp.csr_matrix:
    """P[i, j] = phi^{coarse}_j(x_i) for active fine DoFs i, active coarse DoFs j."""
    x1 = fine.node_coord_1d()
    rows, cols, vals = [], [], []
    for node in map(tuple, np.argwhere(fine.node_active)):
        i = fine.dof_of_node[node]
        x = np.array([x1[I] for I in node])
        for cell in _coarse_cells_containing(fine, node):
            if coarse.active[cell]:
                lo = coarse.cell_lo(cell)
                xi = (x - lo) / coarse.h
                v = eval_tensor_basis(coarse.k, xi[None, :])[0]
                D = coarse.cell_dofs(cell)
                v = np.where(np.abs(v) < 1e-12, 0.0, v)
                nz = v != 0.0
                rows.append(np.full(int(nz.sum()), i))
                cols.append(D[nz])
                vals.append(v[nz])
                break
        else:
            raise ValueError("fine DoF outside every active coarse cell (nestedness)")
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.n_dofs, coarse.n_dofs)).tocsr()
