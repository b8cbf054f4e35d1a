"""Background mesh hierarchy, level set, active/cut cells and DoF numbering
(oracle; test infrastructure only).

Follows the paper, Section 2.1: nested Cartesian meshes M_0 < M_1 < ... < M_L,
the set M_{l,Omega} of cells meeting Omega ("active") and M_{l,Gamma} of cells
meeting the boundary ("cut"); DoFs only on active cells (Section 3, first
paragraph).  Omega is a union of axis-aligned ellipsoids (a sphere is an
ellipsoid with equal semi-axes):

    Omega = { x : min_i q_i(x) < 0 },  q_i(x) = sum_j ((x_j - c_ij)/s_ij)^2 - 1.

Classification of a closed cell box B (strict inequalities, which decide the
measure-zero tangencies):
  * active  iff  min_i min_{x in B} q_i(x) < 0   (the box meets the open set),
  * inside  iff  max_{x in B} q_i(x) < 0 for some i (box inside one shape),
  * cut     iff  active and not inside.
For a single shape this is the exact classification; for unions, a box covered
only jointly by several shapes counts as cut.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from .basis import gll_nodes


@dataclass(frozen=True)
class Shape:
    """Axis-aligned ellipsoid sum_j ((x_j - c_j)/s_j)^2 < 1."""

    center: tuple
    semi: tuple

    @property
    def dim(self) -> int:
        return len(self.center)

    def q(self, x: np.ndarray) -> np.ndarray:
        c = np.asarray(self.center)
        s = np.asarray(self.semi)
        return np.sum(((x - c) / s) ** 2, axis=-1) - 1.0

    def box_min_q(self, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
        """Exact min of q over boxes [lo, hi] (arrays (..., d)); separable."""
        c = np.asarray(self.center)
        s = np.asarray(self.semi)
        dist = np.maximum(np.maximum(lo - c, c - hi), 0.0)
        return np.sum((dist / s) ** 2, axis=-1) - 1.0

    def box_max_q(self, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
        """Exact max of q over boxes (attained at a corner; separable)."""
        c = np.asarray(self.center)
        s = np.asarray(self.semi)
        far = np.maximum(np.abs(lo - c), np.abs(hi - c))
        return np.sum((far / s) ** 2, axis=-1) - 1.0


def sphere(center, radius) -> Shape:
    return Shape(tuple(float(v) for v in center), tuple(float(radius) for _ in center))


@dataclass
class Level:
    """One Cartesian level: N cells per direction on [lo, hi]^d."""

    dim: int
    k: int
    N: int
    lo: float
    hi: float
    active: np.ndarray = field(repr=False, default=None)  # bool, shape (N,)*d, index order (x, y[, z])
    cut: np.ndarray = field(repr=False, default=None)
    node_active: np.ndarray = field(repr=False, default=None)  # bool, shape (kN+1,)*d
    dof_of_node: np.ndarray = field(repr=False, default=None)  # int, -1 where inactive
    n_dofs: int = 0

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.N

    @property
    def n_nodes_1d(self) -> int:
        return self.k * self.N + 1

    def node_coord_1d(self) -> np.ndarray:
        """Coordinates of the 1-D lattice of nodes: cell c, local GLL node a ->
        lattice index k*c + a."""
        xi = gll_nodes(self.k)
        out = np.empty(self.n_nodes_1d)
        for c in range(self.N):
            for a in range(self.k + 1):
                out[self.k * c + a] = self.lo + (c + xi[a]) * self.h
        out[-1] = self.hi
        return out

    def cell_lo(self, cell: tuple) -> np.ndarray:
        return self.lo + np.asarray(cell, dtype=np.float64) * self.h

    def cell_nodes(self, cell: tuple) -> list:
        """Lattice multi-indices of the (k+1)^d nodes of a cell, local order x fastest."""
        k, d = self.k, self.dim
        out = []
        for loc in range((k + 1) ** d):
            a = [(loc // (k + 1) ** i) % (k + 1) for i in range(d)]
            out.append(tuple(k * cell[i] + a[i] for i in range(d)))
        return out

    def cell_dofs(self, cell: tuple) -> np.ndarray:
        return np.array([self.dof_of_node[n] for n in self.cell_nodes(cell)], dtype=np.int64)

    def active_cells(self) -> list:
        return [tuple(int(v) for v in c) for c in np.argwhere(self.active)]

    def dof_coords(self) -> np.ndarray:
        """Coordinates of the active DoFs in canonical order (shape (n, d))."""
        x1 = self.node_coord_1d()
        idx = np.argwhere(self.node_active)
        # canonical order: lexicographic with x fastest
        order = np.lexsort(tuple(idx[:, i] for i in range(self.dim)))
        idx = idx[order]
        return np.stack([x1[idx[:, i]] for i in range(self.dim)], axis=1)


def classify_cells(shapes, dim: int, N: int, lo: float, hi: float):
    """Active and cut masks of all N^d cells (index order x, y[, z])."""
    h = (hi - lo) / N
    grids = np.meshgrid(*[np.arange(N)] * dim, indexing="ij")
    cidx = np.stack(grids, axis=-1).astype(np.float64)
    blo = lo + cidx * h
    bhi = lo + (cidx + 1.0) * h
    active = np.zeros((N,) * dim, dtype=bool)
    inside = np.zeros((N,) * dim, dtype=bool)
    for s in shapes:
        active |= s.box_min_q(blo, bhi) < 0.0
        inside |= s.box_max_q(blo, bhi) < 0.0
    return active, active & ~inside


def number_dofs(level: Level) -> None:
    """Mark lattice nodes lying in the closure of at least one active cell and
    number them in canonical order (lexicographic, x fastest)."""
    k, d, N = level.k, level.dim, level.N
    nn = level.n_nodes_1d
    node_active = np.zeros((nn,) * d, dtype=bool)
    for cell in np.argwhere(level.active):
        sl = tuple(slice(k * int(c), k * int(c) + k + 1) for c in cell)
        node_active[sl] = True
    level.node_active = node_active
    dof = -np.ones((nn,) * d, dtype=np.int64)
    idx = np.argwhere(node_active)
    order = np.lexsort(tuple(idx[:, i] for i in range(d)))
    idx = idx[order]
    dof[tuple(idx.T)] = np.arange(len(idx))
    level.dof_of_node = dof
    level.n_dofs = len(idx)


def build_levels(shapes, dim: int, k: int, n_levels: int, coarse_cells: int, lo: float, hi: float):
    """Level hierarchy l = 0..n_levels-1 with N_l = coarse_cells * 2^l.

    Checks the nestedness Omega_l within Omega_{l-1} required by the embedding
    prolongation (paper, Section 2.2): every active cell must have an active parent.
    """
    levels = []
    for l in range(n_levels):
        N = coarse_cells * 2 ** l
        active, cut = classify_cells(shapes, dim, N, lo, hi)
        lev = Level(dim=dim, k=k, N=N, lo=lo, hi=hi, active=active, cut=cut)
        number_dofs(lev)
        if l > 0:
            parent = levels[-1].active
            for cell in np.argwhere(active):
                if not parent[tuple(int(c) // 2 for c in cell)]:
                    raise ValueError("nestedness violated: active cell with inactive parent")
        levels.append(lev)
    if levels[0].n_dofs == 0:
        raise ValueError("no active cells on the coarsest level")
    return levels


def neighbours(cell: tuple, N: int):
    """Face neighbours (direction, +1 side) of a cell inside the background box."""
    for i in range(len(cell)):
        if cell[i] + 1 < N:
            nb = list(cell)
            nb[i] += 1
            yield i, tuple(nb)


def cell_offsets(dim: int):
    return list(itertools.product((0, 1), repeat=dim))
