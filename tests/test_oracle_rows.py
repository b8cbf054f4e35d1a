"""The one-row-at-a-time oracle of the full-size GPU tests (tests/oracle_rows.py)
against the oracle's whole-level assembly and patch sets on small levels: every
row, every patch class and the union of every colour's internal nodes."""
import numpy as np
import pytest

import workloads as W
from oracle_rows import OracleRows


@pytest.mark.parametrize("w", [W.disc_union(2, 3), W.offcentre_ball(2, 3), W.offcentre_ball(3, 2)], ids=lambda w: w.name)
def test_rows_and_patches_match_the_whole_level(w):
    from oracle.assemble import assemble
    from oracle.multigrid import build_patches

    R = OracleRows(w)
    A = assemble(R.L, R.shapes, R.fp).tocsr()
    for i in range(R.L.n_dofs):
        cols, vals = R.row(i)
        ref = A[i].toarray().ravel()
        got = np.zeros_like(ref)
        got[cols] = vals
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), i
    groups = build_patches(R.L, A)
    for colour in range(2 ** w.dim):
        cut_v, int_v = R.patch_masks(colour)
        for interior, vm in ((False, cut_v), (True, int_v)):
            ps = groups.get((interior, colour))
            want = sorted(ps.vertices) if ps else []
            assert sorted(tuple(int(t) for t in v) for v in np.argwhere(vm)) == want, (interior, colour)
            dofs = R.L.dof_of_node[R.internal_node_mask(vm)]
            union = np.unique(np.concatenate(ps.dofs)) if ps else np.zeros(0, dtype=np.int64)
            assert np.array_equal(np.unique(dofs[dofs >= 0]), union), (interior, colour)
