"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only describes inputs: domain geometry, discretisation parameters
and seeded random vectors.  It holds none of the method's arithmetic.

Domains follow the benchmark configurations of the method's evaluation: a disc
or a ball of radius 0.7 cut from the background box [-1, 1]^d, a union of
seeded spheres, all on a 4^d coarse Cartesian mesh refined uniformly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    k: int                      # polynomial degree
    n_levels: int               # levels 0..n_levels-1, N_l = coarse_cells * 2^l
    coarse_cells: int = 4
    lo: float = -1.0
    hi: float = 1.0
    centers: tuple = ()         # one tuple of length dim per shape
    semi: tuple = ()            # semi-axes per shape (all equal for a sphere)
    gamma_g: float = 0.1        # ghost penalty for every derivative order
    gamma_m: tuple = ()         # per derivative order m = 1.. (overrides gamma_g where given)
    ghost_exp_mode: int = 0     # 0: h^(2m-1) scaling, 1: h^(2m+1)
    n_c: int = 2                # sweeps over the cut patches per smoothing step
    rhs: str = "manufactured"   # "manufactured" (u = prod sin(pi x_j)) or "fourier"
    nrhs: int = 1

    @property
    def gamma_D(self) -> float:
        """Nitsche penalty; the penalty term reads gamma_D / h with gamma_D = 20 k (k+1)."""
        return 20.0 * self.k * (self.k + 1)

    @property
    def fine_cells(self) -> int:
        return self.coarse_cells * 2 ** (self.n_levels - 1)

    def with_levels(self, n_levels: int) -> "Workload":
        return Workload(**{**self.__dict__, "n_levels": n_levels,
                           "name": f"{self.name}@{self.coarse_cells * 2 ** (n_levels - 1)}"})

    def with_degree(self, k: int) -> "Workload":
        return Workload(**{**self.__dict__, "k": k, "name": f"{self.name}-Q{k}"})


def disc_q2() -> Workload:
    """2-D disc |x| < 0.7 in [-1, 1]^2, Q2, 4 levels (4x4 to 32x32 cells)."""
    return Workload("disc-r0.7-Q2", 2, 2, 4, centers=((0.0, 0.0),), semi=((0.7, 0.7),))


def ball_q2() -> Workload:
    """3-D ball |x| < 0.7 in [-1, 1]^3, Q2, 6 levels (4^3 to 128^3 cells)."""
    return Workload("ball-r0.7-Q2", 3, 2, 6, centers=((0.0, 0.0, 0.0),), semi=((0.7, 0.7, 0.7),))


def offcentre_disc(k: int = 2, n_levels: int = 4) -> Workload:
    """A disc that is not symmetric w.r.t. the mesh, to exercise generic cuts."""
    return Workload(f"disc-off-Q{k}", 2, k, n_levels, centers=((0.0731, -0.1123),), semi=((0.6613, 0.6613),))


def offcentre_ball(k: int = 2, n_levels: int = 3) -> Workload:
    return Workload(f"ball-off-Q{k}", 3, k, n_levels, centers=((0.0513, -0.0821, 0.0337),),
                    semi=((0.6471, 0.6471, 0.6471),))


def ellipse(k: int = 2, n_levels: int = 4) -> Workload:
    return Workload(f"ellipse-Q{k}", 2, k, n_levels, centers=((0.031, -0.047),), semi=((0.72, 0.51),))


def box_disc(k: int = 2, n_levels: int = 4) -> Workload:
    """A disc of radius 1.3 around the origin: it covers [-1, 1]^2 except the
    corners, so the operator tiles along the box edges are regular up to the
    box (the last owned layer of the last tile included)."""
    return Workload(f"box-disc-Q{k}", 2, k, n_levels, centers=((0.0, 0.0),), semi=((1.3, 1.3),))


def box_ball(k: int = 2, n_levels: int = 3) -> Workload:
    """The 3-D counterpart of box_disc (radius 1.3 in [-1, 1]^3)."""
    return Workload(f"box-ball-Q{k}", 3, k, n_levels, centers=((0.0, 0.0, 0.0),), semi=((1.3, 1.3, 1.3),))


def disc_union(k: int = 2, n_levels: int = 3) -> Workload:
    """Two overlapping discs (union)."""
    return Workload(f"disc-union-Q{k}", 2, k, n_levels, centers=((-0.21, 0.05), (0.27, -0.11)),
                    semi=((0.45, 0.45), (0.38, 0.38)))


def ball_union(k: int = 2, n_levels: int = 3) -> Workload:
    """Two overlapping balls (union)."""
    return Workload(f"ball-union-Q{k}", 3, k, n_levels, centers=((-0.19, 0.04, 0.02), (0.25, -0.09, -0.05)),
                    semi=((0.46, 0.46, 0.46), (0.37, 0.37, 0.37)))


def sphere_union_8(k: int = 3, n_levels: int = 5, seed: int = 0) -> Workload:
    """Union of 8 spheres in [-1, 1]^3 with centres uniform in [-0.6, 0.6]^3 and radii
    uniform in [0.15, 0.35], both drawn from default_rng(seed) (centres first)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.6, 0.6, (8, 3))
    radii = rng.uniform(0.15, 0.35, 8)
    return Workload(f"sphere-union8-s{seed}-Q{k}", 3, k, n_levels,
                    centers=tuple(tuple(float(v) for v in c) for c in centres),
                    semi=tuple((float(r),) * 3 for r in radii))


def paper_circle(k: int, L: int, n_c: int = 2) -> Workload:
    """The paper's 2-D protocol: circle of radius 1 around the origin in the box
    [-1.105, 1.105]^2 (the half-width that reproduces the paper's DoF counts),
    2x2 coarsest cells, finest level L (2^(L+1) cells per direction), n_c sweeps
    over the cut patches."""
    return Workload(f"circle-paper-Q{k}-L{L}-nc{n_c}", 2, k, L + 1, coarse_cells=2, lo=-1.105, hi=1.105,
                    centers=((0.0, 0.0),), semi=((1.0, 1.0),), n_c=n_c)


def shape_family(n: int, seed: int = 0, dim: int = 3, k: int = 2, n_levels: int = 4) -> list:
    """n geometries of one lattice shape (same dim, k, levels, box): each an
    ellipsoid with centre in U[-0.2, 0.2]^d and semi-axes in U[0.45, 0.7], or
    (probability 1/2) the union of two such ellipsoids with semi-axes in
    U[0.35, 0.55] and centres in U[-0.3, 0.3]^d, drawn from default_rng(seed).
    Large enough that every colour of every level has cut patches."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        m = 1 if rng.random() < 0.5 else 2
        c, lo, hi = (0.2, 0.45, 0.7) if m == 1 else (0.3, 0.35, 0.55)
        centers = tuple(tuple(float(v) for v in rng.uniform(-c, c, dim)) for _ in range(m))
        semi = tuple(tuple(float(v) for v in rng.uniform(lo, hi, dim)) for _ in range(m))
        out.append(Workload(f"family{seed}-{i}-d{dim}-m{m}-Q{k}-N{4 * 2 ** (n_levels - 1)}", dim, k, n_levels,
                            centers=centers, semi=semi))
    return out


def random_vector(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """Seeded standard-normal test vector(s), float64, shape (n,) or (nrhs, n)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nrhs, n))
    return v[0] if nrhs == 1 else v


def fourier_modes(dim: int, seed: int, n_modes: int = 16):
    """Seeded random smooth Fourier data for f = sum_q a_q cos(pi kappa_q . x + theta_q):
    kappa_q drawn from {0..4}^d without the zero vector, a_q ~ N(0,1) / (1 + |kappa_q|^2),
    theta_q ~ U[0, 2 pi).  Returns (kappa (n_modes, dim) int32, a, theta)."""
    rng = np.random.default_rng(seed)
    kappa = np.zeros((n_modes, dim), dtype=np.int32)
    for q in range(n_modes):
        while True:
            kq = rng.integers(0, 5, size=dim)
            if kq.any():
                break
        kappa[q] = kq
    amp = rng.standard_normal(n_modes) / (1.0 + np.sum(kappa.astype(np.float64) ** 2, axis=1))
    theta = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    return kappa, amp, theta


def serving_stream(n_requests: int, seed: int = 0, pool: int = 32, zipf_a: float = 1.1,
                   fine_cells=(32, 64, 128), degrees=(1, 2, 3), dims=(2, 3), max_dofs: int = None,
                   max_shapes: int = 4):
    """Seeded request stream for the solve server.

    A pool of `pool` geometries is drawn first: dimension d, a union of m shapes
    with m uniform in 1..max_shapes, each a sphere or an axis-aligned ellipsoid
    (probability 1/2 each) with centre in U[-0.5, 0.5]^d and radius / semi-axes
    in U[0.2, 0.5] (m = 1) or U[0.15, 0.4] (m > 1), degree k, fine mesh N_L
    with levels = log2(N_L / 4) + 1.  Each request picks a pool entry with
    Zipf(zipf_a) popularity and its own random Fourier right-hand side (seed
    1000 + request index).  Returns a list of (workload, (kappa, amp, theta))
    pairs.  max_dofs drops pool entries whose background lattice exceeds it
    (bounded runs)."""
    rng = np.random.default_rng(seed)
    entries = []
    while len(entries) < pool:
        d = int(rng.choice(dims))
        k = int(rng.choice(degrees))
        NL = int(rng.choice(fine_cells))
        m = int(rng.integers(1, max_shapes + 1))
        lo, hi = (0.2, 0.5) if m == 1 else (0.15, 0.4)
        centers, semi = [], []
        for _ in range(m):
            centers.append(tuple(float(v) for v in rng.uniform(-0.5, 0.5, d)))
            if rng.random() < 0.5:
                semi.append((float(rng.uniform(lo, hi)),) * d)
            else:
                semi.append(tuple(float(v) for v in rng.uniform(lo, hi, d)))
        if max_dofs is not None and (k * NL + 1) ** d > max_dofs:
            continue
        levels = int(np.log2(NL // 4)) + 1
        entries.append(Workload(f"pool{len(entries)}-d{d}-m{m}-Q{k}-N{NL}", d, k, levels, centers=tuple(centers),
                                semi=tuple(semi), rhs="fourier"))
    ranks = np.arange(1, pool + 1, dtype=np.float64)
    prob = ranks ** (-zipf_a)
    prob /= prob.sum()
    out = []
    for i in range(n_requests):
        w = entries[int(rng.choice(pool, p=prob))]
        out.append((w, fourier_modes(w.dim, 1000 + i)))
    return out
