"""Build the whole discrete problem of a workload (oracle; test infrastructure only)."""
from __future__ import annotations

import math

import numpy as np

from .assemble import FormParams, assemble, load_vector
from .geometry import Shape, build_levels
from .multigrid import Hierarchy
from .transfer import prolongation


def shapes_of(w) -> list:
    return [Shape(tuple(c), tuple(s)) for c, s in zip(w.centers, w.semi)]


def form_params(w) -> FormParams:
    return FormParams(gamma_D=w.gamma_D, gamma_g=w.gamma_g, ghost_exp_mode=w.ghost_exp_mode, gamma_m=tuple(w.gamma_m))


def manufactured(dim: int):
    """u = prod_j sin(pi x_j), f = -Laplace u = dim pi^2 u, Dirichlet data g = u."""
    u = lambda x: np.prod(np.sin(math.pi * x), axis=-1)
    f = lambda x: dim * math.pi ** 2 * u(x)
    return u, f, u


def build(w, with_hierarchy: bool = True, dtype=np.float64, n_levels: int = None):
    """Levels, matrices A_l, prolongations and (optionally) the multigrid hierarchy."""
    shapes = shapes_of(w)
    fp = form_params(w)
    L = w.n_levels if n_levels is None else n_levels
    levels = build_levels(shapes, w.dim, w.k, L, w.coarse_cells, w.lo, w.hi)
    mats = [assemble(lev, shapes, fp) for lev in levels]
    prols = [prolongation(levels[l - 1], levels[l]) for l in range(1, L)]
    hier = Hierarchy(levels, mats, prols, n_c=w.n_c, dtype=dtype) if with_hierarchy else None
    return levels, mats, prols, hier


def rhs(w, level):
    u, f, g = manufactured(w.dim)
    return load_vector(level, shapes_of(w), form_params(w), f, g)


def fourier_f(kappa, amp, theta):
    """f(x) = sum_q a_q cos(pi kappa_q . x + theta_q)."""
    kappa = np.asarray(kappa, dtype=np.float64)

    def f(x):
        return np.cos(math.pi * x @ kappa.T + theta) @ amp

    return f


def rhs_fourier(w, level, kappa, amp, theta):
    """Load vector of the Fourier data with homogeneous Dirichlet data."""
    return load_vector(level, shapes_of(w), form_params(w), fourier_f(kappa, amp, theta), None)
