"""Pins of the cut-cell quadrature against closed forms of discs, balls and ellipses."""
import math

import numpy as np
import pytest
from scipy.special import ellipe

from oracle.geometry import Shape, classify_cells, sphere
from oracle.quadrature import cut_cell_rule


def _integrate(shape, d, N, lo=-1.0, hi=1.0, n=14):
    """Volume, surface, int_Omega x_0^2, int_Gamma x.n, int_Gamma x_0^2 over the whole mesh."""
    act, cut = classify_cells([shape], d, N, lo, hi)
    h = (hi - lo) / N
    V = S = M2 = XN = G2 = 0.0
    for c in np.argwhere(cut):
        a = lo + c * h
        vx, vw, sx, sw, sn = cut_cell_rule(shape, a, a + h, n=n, n_t=4)
        V += vw.sum()
        M2 += (vw * vx[:, 0] ** 2).sum()
        S += sw.sum()
        XN += (sw * np.sum(sx * sn, axis=1)).sum()
        G2 += (sw * sx[:, 0] ** 2).sum()
    for c in np.argwhere(act & ~cut):
        a = lo + c * h
        V += h ** d
        M2 += (((a[0] + h) ** 3 - a[0] ** 3) / 3.0) * h ** (d - 1)
    return V, S, M2, XN, G2


@pytest.mark.parametrize("N", [4, 8, 32])
def test_disc_closed_forms(N):
    r = 0.7
    V, S, M2, XN, G2 = _integrate(sphere([0.0, 0.0], r), 2, N)
    assert abs(V / (math.pi * r * r) - 1) < 1e-13
    assert abs(S / (2 * math.pi * r) - 1) < 1e-13
    assert abs(M2 / (math.pi * r ** 4 / 4) - 1) < 1e-13
    assert abs(XN / (2 * math.pi * r * r) - 1) < 1e-13  # divergence theorem
    assert abs(G2 / (math.pi * r ** 3) - 1) < 1e-13


def test_offcentre_disc_on_paper_box():
    c = np.array([0.0731, -0.1123])
    r = 0.6613
    V, S, M2, XN, G2 = _integrate(sphere(c, r), 2, 16, -1.105, 1.105)
    assert abs(V / (math.pi * r * r) - 1) < 1e-13
    assert abs(S / (2 * math.pi * r) - 1) < 1e-13
    assert abs(M2 / (math.pi * r * r * (c[0] ** 2 + r * r / 4)) - 1) < 1e-13


@pytest.mark.parametrize("N", [4, 8])
def test_ball_closed_forms(N):
    r = 0.7
    V, S, M2, XN, G2 = _integrate(sphere([0.0, 0.0, 0.0], r), 3, N)
    assert abs(V / (4 / 3 * math.pi * r ** 3) - 1) < 1e-13
    assert abs(S / (4 * math.pi * r * r) - 1) < 1e-13
    assert abs(M2 / (4 * math.pi * r ** 5 / 15) - 1) < 1e-13
    assert abs(XN / (4 * math.pi * r ** 3) - 1) < 1e-13
    assert abs(G2 / (4 * math.pi * r ** 4 / 3) - 1) < 1e-13


def test_ellipse_area_and_perimeter():
    a, b = 0.72, 0.51
    sh = Shape((0.031, -0.047), (a, b))
    V, S, *_ = _integrate(sh, 2, 8)
    assert abs(V / (math.pi * a * b) - 1) < 1e-13
    perim = 4 * a * ellipe(1 - (b / a) ** 2)
    assert abs(S / perim - 1) < 1e-12


def test_single_cell_circular_segment():
    # cell [0.5, 1.5] x [-0.5, 0.5] cut by the unit circle: area of the segment x > 0.5
    r = 1.0
    vx, vw, sx, sw, sn = cut_cell_rule(sphere([0.0, 0.0], r), np.array([0.5, -0.5]), np.array([1.5, 0.5]))
    th = math.acos(0.5)
    seg = r * r * (th - math.sin(th) * math.cos(th))  # x > 0.5 part of the disc
    # only |y| <= 0.5 belongs to the cell; full segment spans |y| <= sqrt(3)/2, subtract caps
    y0 = 0.5
    cap = 2 * (0.5 * (y0 * math.sqrt(1 - y0 * y0) + math.asin(y0)) - 0.5 * y0)  # int_{-y0}^{y0} (sqrt(1-y^2)-0.5) dy
    assert abs(vw.sum() - cap) < 1e-14
    assert abs(sw.sum() - 2 * math.asin(0.5)) < 1e-14  # arc length for |y| <= 0.5
    assert seg > cap
