"""Pins of the cut-cell quadrature against closed forms of discs, balls and ellipses."""
import math

import numpy as np
import pytest
from scipy.special import ellipe

from oracle.geometry import Shape, classify_cells, sphere
from oracle.quadrature import cut_cell_rule, cut_cell_rule_union


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


# ---------------------------------------------------------------------------
# Unions of shapes: closed forms of two overlapping discs / balls (lens and cap
# formulas), the divergence theorem, and the reduction to the single-shape rule.
# The leaf rule on kinked cells is a fixed rule, not a converged one: measured
# errors are ~1e-7 (area / volume) and ~1e-4 (perimeter / surface), so the
# bounds below are loose enough for it and tight enough that a dropped or
# double-counted interval, a wrong merge or a flipped normal (all O(1e-1)) fail.

def _integrate_union(shapes, d, N, lo=-1.0, hi=1.0):
    act, cut = classify_cells(shapes, d, N, lo, hi)
    h = (hi - lo) / N
    V = S = XN = 0.0
    for c in np.argwhere(cut):
        a = lo + c * h
        vx, vw, sx, sw, sn = cut_cell_rule_union(shapes, a, a + h, n=14, n_t=4)
        V += vw.sum()
        S += sw.sum()
        XN += (sw * np.sum(sx * sn, axis=1)).sum()
    V += np.count_nonzero(act & ~cut) * h ** d
    return V, S, XN


def _two_circles(r1, r2, D):
    a1 = math.acos((D * D + r1 * r1 - r2 * r2) / (2 * D * r1))  # half-angle of circle 1's arc inside circle 2
    a2 = math.acos((D * D + r2 * r2 - r1 * r1) / (2 * D * r2))
    lens = r1 * r1 * a1 + r2 * r2 * a2 - 0.5 * math.sqrt((-D + r1 + r2) * (D + r1 - r2) * (D - r1 + r2) * (D + r1 + r2))
    return math.pi * (r1 * r1 + r2 * r2) - lens, r1 * (2 * math.pi - 2 * a1) + r2 * (2 * math.pi - 2 * a2)


def _two_balls(r1, r2, D):
    lens = math.pi * (r1 + r2 - D) ** 2 * (D * D + 2 * D * r2 - 3 * r2 * r2 + 2 * D * r1 + 6 * r1 * r2
                                           - 3 * r1 * r1) / (12 * D)
    x1 = (D * D + r1 * r1 - r2 * r2) / (2 * D)  # distance from centre 1 to the intersection plane
    x2 = D - x1
    caps = 2 * math.pi * r1 * (r1 - x1) + 2 * math.pi * r2 * (r2 - x2)  # caps hidden inside the other ball
    return 4 / 3 * math.pi * (r1 ** 3 + r2 ** 3) - lens, 4 * math.pi * (r1 * r1 + r2 * r2) - caps


@pytest.mark.parametrize("N", [4, 8, 16])
def test_two_disc_union_closed_forms(N):
    c1, c2, r1, r2 = np.array([-0.21, 0.05]), np.array([0.27, -0.11]), 0.45, 0.38
    A, P = _two_circles(r1, r2, float(np.linalg.norm(c1 - c2)))
    V, S, XN = _integrate_union([sphere(c1, r1), sphere(c2, r2)], 2, N)
    assert abs(V / A - 1) < 1e-6
    assert abs(S / P - 1) < 2e-3
    assert abs(XN / (2 * V) - 1) < 1e-3  # int_Gamma x.n = d |Omega|


def test_two_ball_union_closed_forms():
    c1, c2, r1, r2 = np.array([-0.19, 0.04, 0.02]), np.array([0.25, -0.09, -0.05]), 0.46, 0.37
    Vx, Sx = _two_balls(r1, r2, float(np.linalg.norm(c1 - c2)))
    V, S, XN = _integrate_union([sphere(c1, r1), sphere(c2, r2)], 3, 4)
    assert abs(V / Vx - 1) < 1e-6
    assert abs(S / Sx - 1) < 2e-3
    assert abs(XN / (3 * V) - 1) < 1e-3


def test_union_of_disjoint_shapes_is_exact():
    """Shapes that never share a cell: every cut cell meets one surface, so the
    union rule is the single-shape rule and the totals are sums of closed forms."""
    sh = [sphere([-0.5, -0.45], 0.3), Shape((0.5, 0.45), (0.35, 0.25))]
    V, S, XN = _integrate_union(sh, 2, 8)
    assert abs(V / (math.pi * (0.09 + 0.35 * 0.25)) - 1) < 1e-13
    perim = 2 * math.pi * 0.3 + 4 * 0.35 * ellipe(1 - (0.25 / 0.35) ** 2)
    assert abs(S / perim - 1) < 1e-12


def test_union_of_one_shape_is_the_single_rule():
    sh = Shape((0.031, -0.047), (0.72, 0.51))
    a, b = np.array([0.5, 0.0]), np.array([0.75, 0.25])
    one = cut_cell_rule(sh, a, b, n=14, n_t=3)
    uni = cut_cell_rule_union([sh], a, b, n=14, n_t=3)
    for x, y in zip(one, uni):
        assert np.array_equal(x, y)


def test_nested_shapes_reduce_to_the_outer_one():
    """A shape inside another adds nothing: the union is the outer disc."""
    sh = [sphere([0.0, 0.0], 0.7), sphere([0.1, 0.05], 0.2)]
    V, S, _ = _integrate_union(sh, 2, 8)
    assert abs(V / (math.pi * 0.49) - 1) < 1e-13
    assert abs(S / (2 * math.pi * 0.7) - 1) < 1e-13


def test_union_leaf_rule_converges_to_the_closed_forms():
    """The leaf rule on kinked cells is fixed at bisection depth 4 in the
    set-up; deeper bisection must converge to the exact union (lens formula for
    the area, arcs for the perimeter), which pins the rule itself and not only
    its agreement with a second implementation of it."""
    c1, c2, r1, r2 = np.array([-0.21, 0.05]), np.array([0.27, -0.11]), 0.45, 0.38
    A, P = _two_circles(r1, r2, float(np.linalg.norm(c1 - c2)))
    shapes = [sphere(c1, r1), sphere(c2, r2)]
    N, lo, hi = 8, -1.0, 1.0
    h = (hi - lo) / N
    act, cut = classify_cells(shapes, 2, N, lo, hi)
    errs = {}
    for depth in (4, 8, 10):
        V = np.count_nonzero(act & ~cut) * h * h
        S = 0.0
        for c in np.argwhere(cut):
            a = lo + c * h
            vx, vw, sx, sw, sn = cut_cell_rule_union(shapes, a, a + h, n=14, n_t=4, union_depth=depth)
            V += vw.sum()
            S += sw.sum()
        errs[depth] = (abs(V / A - 1), abs(S / P - 1))
    assert errs[4][0] < 1e-6 and errs[4][1] < 1e-3
    assert errs[8][0] < 1e-9 and errs[10][0] < 1e-10
    assert errs[10][1] < 2e-5 and errs[10][1] < errs[4][1] / 20
