"""Rows of a level's operator and patch sets from the oracle, one at a time
(test infrastructure): for levels too large to assemble whole, the GPU tests
take sampled outputs from these."""
import itertools

import numpy as np


class OracleRows:
    """Rows of one level's operator (default: the finest) assembled one at a
    time from the oracle's uncut-cell, cut-cell and ghost-face matrices (the
    same sums as oracle.assemble.assemble, restricted to the cells and faces at
    one node), and the oracle's patch classes on the whole vertex grid."""

    def __init__(self, w, level=-1):
        from oracle import geometry as G
        from oracle import problem as OP
        from oracle.assemble import ghost_face_matrix, uncut_cell_matrix

        self.shapes = OP.shapes_of(w)
        self.fp = OP.form_params(w)
        self.L = G.build_levels(self.shapes, w.dim, w.k, w.n_levels, w.coarse_cells, w.lo, w.hi)[level]
        L = self.L
        self.k, self.d, self.N = L.k, L.dim, L.N
        self.nloc = (self.k + 1) ** self.d
        self.K = uncut_cell_matrix(self.k, self.d, L.h)
        self.Gf = [ghost_face_matrix(self.k, self.d, L.h, i, self.fp) for i in range(self.d)]
        idx = np.argwhere(L.node_active)
        self.node_of_dof = idx[np.lexsort(tuple(idx[:, i] for i in range(self.d)))]
        self._cut = {}

    def cell_matrix(self, c):
        from oracle.assemble import cut_cell_matrix

        if not self.L.cut[c]:
            return self.K
        if c not in self._cut:
            self._cut[c] = cut_cell_matrix(self.L, self.shapes, c, self.fp)
        return self._cut[c]

    def _local(self, node, c):
        return sum((node[i] - self.k * c[i]) * (self.k + 1) ** i for i in range(self.d))

    def row(self, dof):
        """(columns, values) of row `dof`, duplicates summed."""
        L, k, d, N = self.L, self.k, self.d, self.N
        node = tuple(int(v) for v in self.node_of_dof[dof])
        cand = []
        for i in range(d):
            cs = {node[i] // k}
            if node[i] % k == 0:
                cs.add(node[i] // k - 1)
            cand.append(sorted(c for c in cs if 0 <= c < N))
        cols, vals = [], []
        faces = set()
        for c in itertools.product(*cand):
            if not L.active[c]:
                continue
            cols.append(L.cell_dofs(c))
            vals.append(self.cell_matrix(c)[self._local(node, c)])
            for i in range(d):
                for s in (-1, 1):
                    nb = list(c)
                    nb[i] += s
                    nb = tuple(nb)
                    if 0 <= nb[i] < N and L.active[nb] and (L.cut[c] or L.cut[nb]):
                        faces.add((i, min(c, nb), max(c, nb)))
        for i, lo, hi in faces:
            D = np.concatenate([L.cell_dofs(lo), L.cell_dofs(hi)])
            for side, c in ((0, lo), (1, hi)):
                if all(k * c[j] <= node[j] <= k * c[j] + k for j in range(d)):
                    cols.append(D)
                    vals.append(self.Gf[i][side * self.nloc + self._local(node, c)])
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        u, inv = np.unique(cols, return_inverse=True)
        return u, np.bincount(inv, weights=vals)

    def patch_internal(self, V):
        from oracle.multigrid import patch_internal_dofs

        return patch_internal_dofs(self.L, V)

    def patch_masks(self, colour):
        """Vertex masks of the cut and of the interior patches of one colour
        (the oracle's is_interior_patch, evaluated on the whole vertex grid)."""
        L, d, N = self.L, self.d, self.N
        act = np.pad(L.active, 2)
        cut = np.pad(L.cut, 2)
        has_cell = np.zeros((N + 1,) * d, dtype=bool)
        all_regular = np.ones((N + 1,) * d, dtype=bool)
        ring_cut = np.zeros((N + 1,) * d, dtype=bool)
        # cell V - 1 + off sits at padded index V + 1 + off
        for off in itertools.product((0, 1), repeat=d):
            sl = tuple(slice(1 + o, 1 + o + N + 1) for o in off)
            has_cell |= act[sl]
            all_regular &= act[sl] & ~cut[sl]
            for i in range(d):  # the face neighbour of that cell outside the 2^d box
                o2 = list(off)
                o2[i] = -1 if off[i] == 0 else 2
                ring_cut |= cut[tuple(slice(1 + o, 1 + o + N + 1) for o in o2)]
        interior = all_regular & ~ring_cut
        V = np.indices((N + 1,) * d)
        col = sum((V[i] % 2) << i for i in range(d)) == colour
        return has_cell & ~interior & col, has_cell & interior & col

    def internal_node_mask(self, vmask):
        """Lattice nodes strictly inside the patch boxes of the marked vertices."""
        k, d = self.k, self.d
        nn = k * self.N + 1
        out = np.zeros((nn,) * d, dtype=bool)
        vs = np.argwhere(vmask)
        for off in itertools.product(range(-k + 1, k), repeat=d):
            nodes = k * vs + np.array(off)
            ok = np.all((nodes >= 0) & (nodes < nn), axis=1)
            out[tuple(nodes[ok].T)] = True
        return out
