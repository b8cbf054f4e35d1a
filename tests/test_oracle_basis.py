"""Pins of the oracle's 1-D basis and uncut element matrices against closed forms."""
import math

import numpy as np
import pytest

from oracle.basis import eval_basis, gll_nodes, gauss_legendre
from oracle.assemble import uncut_cell_matrix


def test_gll_nodes_closed_form():
    assert np.allclose(gll_nodes(1), [0.0, 1.0], atol=0, rtol=0)
    assert np.allclose(gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-15)
    r5 = 1.0 / math.sqrt(5.0)
    assert np.allclose(gll_nodes(3), [0.0, (1 - r5) / 2, (1 + r5) / 2, 1.0], atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_lagrange_property_and_partition_of_unity(k):
    V = eval_basis(k, gll_nodes(k))
    assert np.allclose(V, np.eye(k + 1), atol=1e-13)
    t = np.linspace(0, 1, 17)
    assert np.allclose(eval_basis(k, t).sum(axis=1), 1.0, atol=1e-13)
    for m in range(1, k + 1):
        assert np.allclose(eval_basis(k, t, m).sum(axis=1), 0.0, atol=1e-10)


def test_gauss_legendre_exactness():
    x, w = gauss_legendre(4)
    for p in range(8):
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-15


def test_q1_element_matrices():
    h = 0.37
    K1 = uncut_cell_matrix(1, 1, h)
    assert np.allclose(K1, np.array([[1, -1], [-1, 1]]) / h, atol=1e-14)
    # 2-D bilinear stiffness is h-independent: (1/6)[[4,-1,-1,-2],...] in x-fastest order
    K2 = uncut_cell_matrix(1, 2, h)
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.allclose(K2, ref, atol=1e-14)


def test_q2_1d_stiffness():
    h = 0.25
    K = uncut_cell_matrix(2, 1, h)
    assert np.allclose(K, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * h), atol=1e-13)


@pytest.mark.parametrize("k,d", [(1, 3), (2, 2), (2, 3), (3, 2)])
def test_uncut_matrix_kernel_and_scaling(k, d):
    K = uncut_cell_matrix(k, d, 1.0)
    assert np.allclose(K @ np.ones(len(K)), 0.0, atol=1e-12)
    assert np.allclose(K, K.T, atol=1e-14)
    assert np.allclose(uncut_cell_matrix(k, d, 0.5), 0.5 ** (d - 2) * K, atol=1e-12)
