"""One-dimensional building blocks of the Q_k space (oracle; test infrastructure only).

The finite element space on every level is the tensor-product space Q_k with a
nodal basis interpolating at the Gauss-Lobatto points of each cell (paper,
Section 2.1, eq. (spaces) and the sentence after it).  Everything here lives on
the reference interval [0, 1]; physical scaling by the cell size h is applied by
the callers.

Plain, slow and obvious on purpose: Lagrange polynomials are built as numpy
polynomial objects and differentiated symbolically.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


@functools.lru_cache(maxsize=None)
def gll_nodes(k: int) -> np.ndarray:
    """Gauss-Lobatto points of degree k on [0, 1], ascending.

    They are the end points together with the roots of P_k' (derivative of the
    Legendre polynomial of degree k), mapped from [-1, 1] to [0, 1].
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    coef = np.zeros(k + 1)
    coef[k] = 1.0
    inner = npleg.legroots(npleg.legder(coef)) if k >= 2 else np.zeros(0)
    t = np.concatenate(([-1.0], np.sort(inner.real), [1.0]))
    return (t + 1.0) / 2.0


@functools.lru_cache(maxsize=None)
def gauss_legendre(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Legendre rule on [0, 1] (exact for degree 2n-1)."""
    x, w = npleg.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


@functools.lru_cache(maxsize=None)
def lagrange_coeffs(k: int) -> np.ndarray:
    """Monomial coefficients of the k+1 Lagrange polynomials on the GLL nodes.

    Row a holds c with psi_a(t) = sum_p c[p] t^p and psi_a(node_b) = delta_ab.
    """
    nodes = gll_nodes(k)
    out = np.zeros((k + 1, k + 1))
    for a in range(k + 1):
        poly = np.array([1.0])
        denom = 1.0
        for b in range(k + 1):
            if b == a:
                continue
            poly = nppoly.polymul(poly, np.array([-nodes[b], 1.0]))
            denom *= nodes[a] - nodes[b]
        out[a, : len(poly)] = poly / denom
    return out


def eval_basis(k: int, t: np.ndarray, deriv: int = 0) -> np.ndarray:
    """Values of the deriv-th derivative (in the reference variable) of all
    k+1 one-dimensional basis functions at the points t.  Shape (len(t), k+1)."""
    t = np.asarray(t, dtype=np.float64)
    c = lagrange_coeffs(k)
    out = np.empty(t.shape + (k + 1,))
    for a in range(k + 1):
        p = c[a]
        for _ in range(deriv):
            p = nppoly.polyder(p)
        out[..., a] = nppoly.polyval(t, p) if len(p) else 0.0
    return out


def local_index_tuples(k: int, d: int) -> np.ndarray:
    """Multi-indices (a_0, ..., a_{d-1}) of the (k+1)^d cell-local basis
    functions in local order, x fastest: local = a_0 + (k+1) a_1 + (k+1)^2 a_2."""
    n = k + 1
    idx = np.arange(n ** d)
    return np.stack([(idx // n ** i) % n for i in range(d)], axis=1)


def eval_tensor_basis(k: int, xi: np.ndarray, deriv_dirs=None) -> np.ndarray:
    """Tensor-product basis on the reference cell at points xi (shape (P, d)).

    deriv_dirs: None for values, or an int i for the first derivative in
    reference direction i.  Returns shape (P, (k+1)^d).
    """
    xi = np.atleast_2d(xi)
    d = xi.shape[1]
    tup = local_index_tuples(k, d)
    out = np.ones((xi.shape[0], tup.shape[0]))
    for i in range(d):
        order = 1 if (deriv_dirs is not None and deriv_dirs == i) else 0
        vals = eval_basis(k, xi[:, i], order)  # (P, k+1)
        out *= vals[:, tup[:, i]]
    return out
