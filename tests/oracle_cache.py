"""One oracle build per workload and test session (test infrastructure).

The oracle is slow on unions of spheres with Q3 (its cut-cell rule runs in
Python); GPU test modules that use the same workload share one build."""
from __future__ import annotations

import functools


@functools.lru_cache(maxsize=8)
def build(w):
    from oracle import problem as OP

    return OP.build(w)


@functools.lru_cache(maxsize=8)
def hierarchy32(w):
    import numpy as np

    from oracle.multigrid import Hierarchy

    levels, mats, prols, _ = build(w)
    return Hierarchy(levels, mats, prols, n_c=w.n_c, dtype=np.float32)
