"""Vertex patches, the coloured multiplicative vertex-patch smoother, the V-cycle
and preconditioned CG (oracle; test infrastructure only).

Paper, Section 2.3 and Section 3:
  * Vertex patches: the cells around a vertex X_j; the patch space V_{l,j}
    holds the basis functions supported in the patch ("internal DoFs"), the
    local matrix A_{l,j} is the principal submatrix of A_l on them.
  * Local solver, eq. (local-solver): correction Q_j^T A_j^{-1} Q_j (b - A x).
  * MVS, eq. (smoother): patch corrections applied one after the other.  The
    printed recursion drops the previous iterate and flips the sign of the
    residual; the reading used here is y_j = y_{j-1} + Q_j^T A_j^{-1} Q_j (b - A y_{j-1}).
  * Colouring: same-coloured patches have disjoint interiors and are applied
    simultaneously, each from the state at the start of the colour step; the
    ghost-penalty coupling between same-coloured patches is ignored (the
    "inconsistent" parallel smoother).  The residual itself is exact.
  * Split smoother, eq. (smoother-split): interior patches first, then n_c
    sweeps over the cut patches; interior patches use the Cartesian patch
    Laplacian (fast diagonalisation in the paper), cut patches a dense inverse
    of the exact principal submatrix.
  * V-cycle with one pre- and one post-smoothing step and an exact coarse
    solve (Section 2.2 and Section 4); the post-smoother runs the colour steps
    of the pre-smoother in reverse order, so the V-cycle is symmetric.
Readings where the paper is not explicit:
  * patch centres are all vertices of active cells (truncated patches at the
    boundary of Omega_l), so that every DoF lies in some patch;
  * a patch is "interior" when its local matrix, the principal submatrix of
    A_l (Section 2.3), is exactly the Cartesian patch Laplacian: all 2^d cells
    exist, are active and uncut, and no ghost face lies on the patch boundary.
    Every other patch is a "cut" patch with a dense inverse.  (Treating
    patches next to a ghost face as Cartesian makes the Q3 colour steps
    divergent, so the paper's definition of A_{l,j} is kept exact here.)
  * colour of vertex X with integer coordinates V: sum_i (V_i mod 2) 2^i.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assemble import uncut_cell_matrix
from .geometry import Level


@dataclass
class PatchSet:
    """Patches of one (class, colour) group on one level."""

    interior: bool
    colour: int
    vertices: list = field(default_factory=list)
    dofs: list = field(default_factory=list)      # list of int arrays (internal DoFs)
    invs: list = field(default_factory=list)      # list of dense local inverses
    rows: np.ndarray = None                        # union of all dofs (sorted)
    closures: list = field(default_factory=list)  # list of int arrays (DoFs of the closed patch box)


def patch_vertices(level: Level) -> list:
    """All vertices of active cells, lexicographic with x fastest."""
    d = level.dim
    verts = set()
    for c in level.active_cells():
        for off in itertools.product((0, 1), repeat=d):
            verts.add(tuple(c[i] + off[i] for i in range(d)))
    return sorted(verts, key=lambda v: tuple(reversed(v)))


def patch_cells(level: Level, V: tuple) -> list:
    d, N = level.dim, level.N
    out = []
    for off in itertools.product((0, 1), repeat=d):
        c = tuple(V[i] - 1 + off[i] for i in range(d))
        if all(0 <= c[i] < N for i in range(d)):
            out.append(c)
    return out


def patch_internal_dofs(level: Level, V: tuple) -> np.ndarray:
    """Active DoFs strictly inside the open box (X - h, X + h)^d, lattice order x fastest."""
    k, d = level.k, level.dim
    nn = level.n_nodes_1d
    ranges = [range(max(k * v - k + 1, 0), min(k * v + k - 1, nn - 1) + 1) for v in V]
    out = []
    for node in itertools.product(*reversed(ranges)):
        node = tuple(reversed(node))
        dof = level.dof_of_node[node]
        if dof >= 0:
            out.append(dof)
    return np.array(out, dtype=np.int64)


def patch_closure_dofs(level: Level, V: tuple) -> np.ndarray:
    """Active DoFs in the closed box [X - h, X + h]^d (the nodes of the patch's cells)."""
    k = level.k
    nn = level.n_nodes_1d
    ranges = [range(max(k * v - k, 0), min(k * v + k, nn - 1) + 1) for v in V]
    out = []
    for node in itertools.product(*reversed(ranges)):
        dof = level.dof_of_node[tuple(reversed(node))]
        if dof >= 0:
            out.append(dof)
    return np.array(out, dtype=np.int64)


def is_interior_patch(level: Level, V: tuple, cells: list) -> bool:
    """A patch is interior when its local matrix is exactly the Cartesian
    Laplacian: all 2^d cells exist, are active and are uncut, and no face on the
    patch boundary is a ghost face (no cut cell across it)."""
    d, N = level.dim, level.N
    if len(cells) != 2 ** d or not all(level.active[c] and not level.cut[c] for c in cells):
        return False
    for c in cells:
        for i in range(d):
            # outward neighbour across the patch boundary in direction i
            nb = list(c)
            nb[i] += 1 if c[i] == V[i] else -1
            if 0 <= nb[i] < N and level.cut[tuple(nb)]:
                return False
    return True


def cartesian_patch_laplacian(k: int, d: int, h: float) -> np.ndarray:
    """Stiffness matrix of the 2^d uncut cells of a full patch restricted to its
    (2k-1)^d internal nodes (no Nitsche or ghost terms)."""
    n1 = 2 * k + 1
    Kc = uncut_cell_matrix(k, d, h)
    Ap = np.zeros((n1 ** d, n1 ** d))
    tup = [[(loc // (k + 1) ** i) % (k + 1) for i in range(d)] for loc in range((k + 1) ** d)]
    for off in itertools.product((0, 1), repeat=d):
        idx = [sum((k * off[i] + t[i]) * n1 ** i for i in range(d)) for t in tup]
        Ap[np.ix_(idx, idx)] += Kc
    inner = [sum(t[i] * n1 ** i for i in range(d))
             for t in (list(reversed(p)) for p in itertools.product(range(1, 2 * k), repeat=d))]
    return Ap[np.ix_(inner, inner)]


def build_patches(level: Level, A: sp.csr_matrix, require_spd: bool = True) -> dict:
    """(interior?, colour) -> PatchSet for one level.  require_spd=False admits
    indefinite cut-patch matrices (only for algebraic identities in tests)."""
    k, d = level.k, level.dim
    Ainv_int = np.linalg.inv(cartesian_patch_laplacian(k, d, level.h))
    groups = {}
    Ad = None
    for V in patch_vertices(level):
        cells = patch_cells(level, V)
        interior = is_interior_patch(level, V, cells)
        colour = sum((V[i] % 2) << i for i in range(d))
        dofs = patch_internal_dofs(level, V)
        if interior:
            inv = Ainv_int
        else:
            Aj = A[dofs][:, dofs].toarray()
            w, Q = np.linalg.eigh(Aj)
            if require_spd and w[0] <= 0.0:
                raise np.linalg.LinAlgError("local matrix of a cut patch is not positive definite")
            inv = (Q / w) @ Q.T
        ps = groups.setdefault((interior, colour), PatchSet(interior=interior, colour=colour))
        ps.vertices.append(V)
        ps.dofs.append(dofs)
        ps.invs.append(inv)
        ps.closures.append(patch_closure_dofs(level, V))
    for ps in groups.values():
        ps.rows = np.unique(np.concatenate(ps.dofs))
    return groups


class Hierarchy:
    """Matrices, transfers, patches and coarse solver of all levels."""

    def __init__(self, levels, mats, prols, n_c=2, dtype=np.float64, require_spd=True, ghost_local=False):
        self.levels = levels
        # False: exact residual b - A x on the patch interior (ghost halos
        # included), the variant that keeps the V-cycle symmetric.  True: each
        # cut patch's residual uses x only on its own closure, i.e. the
        # ghost-face terms that reach beyond the closed patch box are dropped
        # (the coupling through ghost penalties between neighbouring patches is
        # ignored in the residual as well); the V-cycle is then not symmetric.
        self.ghost_local = ghost_local
        self.A = [m.astype(dtype) for m in mats]
        self.P = [None] + [p.astype(dtype) for p in prols]
        self.n_c = n_c
        self.dtype = dtype
        self.patches = [None] + [build_patches(levels[l], mats[l], require_spd) for l in range(1, len(levels))]
        A0 = mats[0].toarray()
        self.coarse_inv = np.linalg.inv(A0).astype(dtype)
        self.coarse_cho = sla.cho_factor(A0) if require_spd else None
        self._row_slices = {}
        self._cast_patches()

    def _cast_patches(self):
        for l in range(1, len(self.levels)):
            for key, ps in self.patches[l].items():
                ps.invs = [inv.astype(self.dtype) for inv in ps.invs]
                self._row_slices[(l, key)] = self.A[l][ps.rows]

    # ---- smoother -------------------------------------------------------
    def schedule(self, l: int, post: bool = False) -> list:
        d = self.levels[l].dim
        C = 2 ** d
        seq = [(True, c) for c in range(C)]
        for _ in range(self.n_c):
            seq += [(False, c) for c in range(C)]
        return list(reversed(seq)) if post else seq

    def colour_step(self, l: int, key, x: np.ndarray, b: np.ndarray) -> None:
        """All patches of one colour class, from the same residual."""
        ps = self.patches[l].get(key)
        if ps is None:
            return
        dx = np.zeros_like(x)
        if self.ghost_local and not ps.interior:
            for dofs, clo, inv in zip(ps.dofs, ps.closures, ps.invs):
                r_j = b[dofs] - self.A[l][dofs][:, clo] @ x[clo]
                dx[dofs] += inv @ r_j
            x += dx
            return
        r_rows = b[ps.rows] - self._row_slices[(l, key)] @ x
        r = np.zeros_like(x)
        r[ps.rows] = r_rows
        for dofs, inv in zip(ps.dofs, ps.invs):
            dx[dofs] += inv @ r[dofs]
        x += dx

    def smooth(self, l: int, x: np.ndarray, b: np.ndarray, post: bool = False) -> None:
        for key in self.schedule(l, post):
            self.colour_step(l, key, x, b)

    # ---- V-cycle --------------------------------------------------------
    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        if self.dtype == np.float64 and self.coarse_cho is not None:
            return sla.cho_solve(self.coarse_cho, b)
        return self.coarse_inv @ b

    def vcycle(self, b: np.ndarray, l: int = None) -> np.ndarray:
        if l is None:
            l = len(self.levels) - 1
        b = b.astype(self.dtype)
        if l == 0:
            return self.coarse_solve(b)
        x = np.zeros_like(b)
        self.smooth(l, x, b, post=False)
        r = b - self.A[l] @ x
        e = self.vcycle(self.P[l].T @ r, l - 1)
        x += self.P[l] @ e
        self.smooth(l, x, b, post=True)
        return x


def pcg(A, b, precond, rtol=1e-8, maxit=200):
    """Preconditioned CG from x0 = 0; stops when ||r||_2 <= rtol ||b||_2.

    Returns (x, iterations, residual history)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, hist
    z = precond(r).astype(np.float64)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        Ap = A @ p
        pAp = p @ Ap
        if not pAp > 0.0:
            raise ArithmeticError("CG breakdown: p^T A p <= 0")
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= rtol:
            return x, it, hist
        z = precond(r).astype(np.float64)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist


def gmres(A, b, precond, rtol=1e-9, restart=30, maxit=500):
    """Right-preconditioned restarted GMRES from x0 = 0 (the paper's outer
    solver, Section 2.2 and Section 4): Arnoldi with modified Gram-Schmidt on
    A B, Givens rotations for the least-squares problem, x = x0 + B V_j y.
    Stops when the GMRES residual norm |g_{j+1}| (equal to ||b - A x||_2 in
    exact arithmetic for right preconditioning) is <= rtol ||b||_2.

    Returns (x, iterations, residual history); iterations counts Arnoldi steps
    (one preconditioner application each)."""
    n = len(b)
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, hist
    it = 0
    while it < maxit:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= rtol * nb:
            return x, it, hist
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        converged = False
        for j in range(restart):
            Z[j] = precond(V[j]).astype(np.float64)
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w -= H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= rtol * nb or it >= maxit:
                converged = abs(g[j + 1]) <= rtol * nb
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x += Z[:j_done].T @ y
        if converged:
            return x, it, hist
    return x, it, hist


def vcycle_iteration(A, b, precond, rtol=1e-9, maxit=500):
    """Multigrid as a stand-alone solver (Section 4, Table 3):
    x_{k+1} = x_k + B (b - A x_k) from x_0 = 0, until ||b - A x_k||_2 <= rtol ||b||_2.

    Returns (x, iterations, residual history); None as iterations when the
    residual grows beyond 1e3 ||b|| (divergence)."""
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, hist
    r = b.copy()
    for it in range(1, maxit + 1):
        x += precond(r).astype(np.float64)
        r = b - A @ x
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= rtol:
            return x, it, hist
        if rel > 1e3:
            return x, None, hist
    return x, maxit, hist
