"""Host bookkeeping of the two-buffer cut colour steps (no GPU): the cut region
and the per-DoF copy flags exported by the library are checked against a brute
force construction from the exported patches, and the two-buffer schedule is
replayed on sets of node versions: every step must read a buffer that is up to
date on the cut region, and an even number of steps must leave the first buffer
equal to the plain in-place result."""
import numpy as np
import pytest

import workloads as W

CASES = [W.disc_q2(), W.offcentre_ball(2, 3), W.disc_union(2, 3), W.offcentre_disc(3, 3)]


def _problem(w):
    from paper_2508_11608_amd import Problem
    return Problem(w, device=False)


def _level_data(P, w, l):
    C = 2 ** w.dim
    nodes = [P.export(l, 32 + c, np.int32) for c in range(C)]
    verts = [P.export(l, 48 + c, np.int32) for c in range(C)]
    nxt = [P.export(l, 56 + c, np.uint8) for c in range(C)]
    region = P.export(l, 64, np.int32)
    active = set(P.export(l, 1, np.int32).tolist())
    N = round(len(P.export(l, 2, np.uint8)) ** (1.0 / w.dim))
    return nodes, verts, nxt, region, active, N


def _present(nodes):
    return [c for c in range(len(nodes)) if len(nodes[c])]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_cut_region_and_copy_flags(w):
    P = _problem(w)
    d, k = w.dim, w.k
    for l in range(1, w.n_levels):
        nodes, verts, nxt, region, active, N = _level_data(P, w, l)
        nn = k * N + 1
        assert np.all(np.diff(region) > 0), "region sorted and unique"
        rset = set(region.tolist())
        assert rset <= active, "region holds active nodes only"
        # every node a cut step reads: closure cells V-1..V and the cells across
        # the patch boundary along one direction (V-2 or V+1), active nodes only
        need = set()
        for c in range(2 ** d):
            for v in verts[c]:
                V = [(int(v) // (N + 1) ** a) % (N + 1) for a in range(d)]
                for off in np.ndindex(*(4,) * d):
                    outer = sum(1 for t in off if t in (0, 3))
                    if outer > 1:
                        continue
                    cell = [V[a] - 2 + off[a] for a in range(d)]
                    if any(ci < 0 or ci >= N for ci in cell):
                        continue
                    for q in np.ndindex(*(k + 1,) * d):
                        I = [k * cell[a] + q[a] for a in range(d)]
                        n = sum(I[a] * nn ** a for a in range(d))
                        if n in active:
                            need.add(n)
        assert need <= rset, f"level {l}: region misses {len(need - rset)} nodes"
        assert rset <= need, f"level {l}: region has {len(rset - need)} nodes no step reads"
        present = _present(nodes)
        for i, c in enumerate(present):
            fwd, bwd = present[(i + 1) % len(present)], present[i - 1]
            assert len(nxt[c]) == len(nodes[c])
            in_f = np.isin(nodes[c], nodes[fwd])
            in_b = np.isin(nodes[c], nodes[bwd])
            assert np.array_equal((nxt[c] & 1) != 0, in_f)
            assert np.array_equal((nxt[c] & 2) != 0, in_b)


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
@pytest.mark.parametrize("post", [False, True])
def test_two_buffer_schedule_replay(w, post):
    """Replay one smoothing pass (n_c sweeps) with node versions: the in-place
    reference T sets the internal DoFs of step i to version i + 1."""
    P = _problem(w)
    for l in range(1, w.n_levels):
        nodes, _, nxt, region, _, _ = _level_data(P, w, l)
        present = _present(nodes)
        seq = [c for _ in range(w.n_c) for c in present]
        if post:
            seq = seq[::-1]
        npp = len(seq) - len(seq) % 2
        if npp == 0:
            continue
        mask = 2 if post else 1
        T = {int(n): 0 for n in region}
        X = [dict(T), {}]
        X[1].update({int(n): X[0][int(n)] for n in region})  # X1 = X0 on the cut region
        for i in range(npp):
            A, B = X[i % 2], X[(i + 1) % 2]
            assert all(A[n] == T[n] for n in T), f"level {l} step {i}: the source buffer is stale"
            own = set(nodes[seq[i]].tolist())
            copied = set()
            if i > 0:
                prev = seq[i - 1]
                copied = {int(n) for n, f in zip(nodes[prev], nxt[prev]) if not (f & mask)}
                assert not (copied & own), "copy blocks and patch blocks write disjoint nodes"
            for n in own:
                B[n] = i + 1
                T[n] = i + 1
            for n in copied:
                B[n] = A[n]
        assert all(X[0][n] == T[n] for n in T), f"level {l}: X0 differs from the in-place result"
