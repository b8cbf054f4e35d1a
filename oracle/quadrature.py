"""Quadrature on cut cells (oracle; test infrastructure only).

The paper generates non-tensor quadrature rules on cut cells upfront on the CPU
(Section 3, third paragraph: substitute quadrature built with Saye's algorithm).
This module implements a dimension-reduction rule of that family for one
axis-aligned ellipsoid q(x) = sum_j ((x_j - c_j)/s_j)^2 - 1 and a box B:

  * A height direction e is chosen in which q is monotone on B (B does not
    straddle the plane x_e = c_e).  Along every vertical line the part of the
    line inside Omega is then one interval with an analytic end point t*(x'),
    integrated with Gauss points.  The boundary point (x', t*(x')) carries the
    surface weight |grad q| / |dq/dx_e| (graph parametrisation of Gamma).
  * The integrand over the base box is smooth except where t* meets the top or
    bottom face of B: the traces of q on those faces, which are again
    axis-aligned ellipses (lower-dimensional quadrics).  The base box is split
    at them: in 2-D at their roots, in 3-D by a second height direction in the
    base and break points where the traces cross the base box edges.
  * A box is bisected in all directions when no admissible direction exists or
    when the distance from the box to the square-root singularity of t* is small
    compared with the box size (quality < beta).

With break points at all kinks the integrands are analytic on every piece, so
the rule converges geometrically in the number n of Gauss points per piece.
Returned rules are in physical coordinates.
"""
from __future__ import annotations

import itertools

import numpy as np

from .basis import gauss_legendre


class Quadric:
    """q(x) = sum_j ((x_j - c_j)/s_j)^2 - kappa on R^m."""

    def __init__(self, c, s, kappa=1.0):
        self.c = np.asarray(c, dtype=np.float64)
        self.s = np.asarray(s, dtype=np.float64)
        self.kappa = float(kappa)

    @property
    def m(self) -> int:
        return len(self.c)

    def value(self, x):
        return np.sum(((x - self.c) / self.s) ** 2, axis=-1) - self.kappa

    def grad(self, x):
        return 2.0 * (x - self.c) / self.s ** 2

    def box_min(self, a, b):
        dist = np.maximum(np.maximum(a - self.c, self.c - b), 0.0)
        return float(np.sum((dist / self.s) ** 2) - self.kappa)

    def box_max(self, a, b):
        far = np.maximum(np.abs(a - self.c), np.abs(b - self.c))
        return float(np.sum((far / self.s) ** 2) - self.kappa)

    def crosses(self, a, b) -> bool:
        return self.box_min(a, b) < 0.0 < self.box_max(a, b)

    def restrict(self, j: int, val: float) -> "Quadric":
        keep = [i for i in range(self.m) if i != j]
        return Quadric(self.c[keep], self.s[keep], self.kappa - ((val - self.c[j]) / self.s[j]) ** 2)

    def roots_1d(self):
        """For m == 1: the (up to two) points where q vanishes."""
        if self.kappa < 0.0:
            return []
        r = self.s[0] * np.sqrt(self.kappa)
        return [self.c[0] - r, self.c[0] + r]


def _side_distance(a, b, c):
    """Distance of [a, b] from the point c if the interval does not straddle it,
    together with the side (+1: interval above c); None when it straddles."""
    if a >= c:
        return a - c, 1.0
    if b <= c:
        return c - b, -1.0
    return None


def _quality(q: Quadric, e: int, dist: float, H: float) -> float:
    """Distance from the box to the singular set of the root t*(x') in units of
    the box size H (lower bound derived from |grad w| <= 2 sqrt(kappa)/s_min)."""
    others = [i for i in range(q.m) if i != e]
    smin = min(q.s[i] for i in others) if others else q.s[e]
    kap = max(q.kappa, 1e-300)
    return (dist / q.s[e]) ** 2 * smin / (2.0 * np.sqrt(kap)) / H


def _best_direction(q: Quadric, a, b, dims, beta):
    """Admissible height direction among dims with the largest quality."""
    H = float(np.max(b - a))
    best = None
    for e in dims:
        sd = _side_distance(a[e], b[e], q.c[e])
        if sd is None:
            continue
        qual = _quality(q, e, sd[0], H)
        if best is None or qual > best[1]:
            best = (e, qual, sd[1])
    if best is None or best[1] < beta:
        return None
    return best


def _gauss_on(lo, hi, n):
    x, w = gauss_legendre(n)
    return lo + (hi - lo) * x, (hi - lo) * w


def _pieces(lo, hi, breaks):
    pts = sorted(float(t) for t in breaks if lo < t < hi)
    edges = [lo] + pts + [hi]
    return [(edges[i], edges[i + 1]) for i in range(len(edges) - 1) if edges[i + 1] > edges[i]]


class Rule:
    """Accumulates volume points/weights and surface points/weights/normals."""

    def __init__(self, d):
        self.d = d
        self.vx, self.vw, self.sx, self.sw, self.sn = [], [], [], [], []

    def add_volume(self, x, w):
        self.vx.append(np.atleast_2d(x))
        self.vw.append(np.atleast_1d(w))

    def add_surface(self, x, w, n):
        self.sx.append(np.atleast_2d(x))
        self.sw.append(np.atleast_1d(w))
        self.sn.append(np.atleast_2d(n))

    def arrays(self):
        d = self.d
        cat = lambda L, shape: np.concatenate(L) if L else np.zeros(shape)
        return (cat(self.vx, (0, d)), cat(self.vw, (0,)), cat(self.sx, (0, d)),
                cat(self.sw, (0,)), cat(self.sn, (0, d)))


def _tensor_box(rule: Rule, a, b, n):
    d = len(a)
    xs, ws = zip(*[_gauss_on(a[i], b[i], n) for i in range(d)])
    grid = np.stack(np.meshgrid(*xs, indexing="ij"), axis=-1).reshape(-1, d)
    wgt = np.ones(1)
    for i in range(d):
        wgt = np.multiply.outer(wgt, ws[i])
    rule.add_volume(grid, wgt.reshape(-1))


def _column(q: Quadric, e, side, ae, be, base_pts, base_w, dims_base, n_t, rule: Rule):
    """Integrate over vertical segments in direction e above the given base
    points (base_pts: (P, d-1) ordered as dims_base)."""
    d = q.m
    P = base_pts.shape[0]
    full = np.zeros((P, d))
    full[:, dims_base] = base_pts
    lo_pt = full.copy()
    lo_pt[:, e] = ae
    hi_pt = full.copy()
    hi_pt[:, e] = be
    qa = q.value(lo_pt)
    qb = q.value(hi_pt)
    w = q.kappa - np.sum(((base_pts - q.c[dims_base]) / q.s[dims_base]) ** 2, axis=1)
    tstar = q.c[e] + side * q.s[e] * np.sqrt(np.maximum(w, 0.0))
    inA = qa < 0.0
    inB = qb < 0.0
    seg_lo = np.where(inA, ae, tstar)
    seg_hi = np.where(inB, be, tstar)
    has = inA | inB
    xt, wt = gauss_legendre(n_t)
    for p in np.nonzero(has)[0]:
        lo_, hi_ = seg_lo[p], seg_hi[p]
        if hi_ <= lo_:
            continue
        pts = np.repeat(full[p : p + 1], n_t, axis=0)
        pts[:, e] = lo_ + (hi_ - lo_) * xt
        rule.add_volume(pts, base_w[p] * (hi_ - lo_) * wt)
    cross = inA != inB
    if np.any(cross):
        idx = np.nonzero(cross)[0]
        sp = full[idx].copy()
        sp[:, e] = tstar[idx]
        g = q.grad(sp)
        gn = np.linalg.norm(g, axis=1)
        rule.add_surface(sp, base_w[idx] * gn / np.abs(g[:, e]), g / gn[:, None])


def _integrate_plan(rule: Rule, q: Quadric, a, b, e, side, n, n_t, beta):
    d = q.m
    dims_base = [i for i in range(d) if i != e]
    Qa = q.restrict(e, a[e])
    Qb = q.restrict(e, b[e])
    ab, bb = a[dims_base], b[dims_base]
    if d == 2:
        breaks = []
        for Q in (Qa, Qb):
            breaks += Q.roots_1d()
        xs, ws = [], []
        for lo_, hi_ in _pieces(ab[0], bb[0], breaks):
            x, w = _gauss_on(lo_, hi_, n)
            xs.append(x)
            ws.append(w)
        base = np.concatenate(xs)[:, None]
        bw = np.concatenate(ws)
        _column(q, e, side, a[e], b[e], base, bw, dims_base, n_t, rule)
        return True
    # d == 3: a 2-D base box with the traces Qa, Qb as kink curves.
    crossing = [Q for Q in (Qa, Qb) if Q.crosses(ab, bb)]
    if crossing:
        Hb = float(np.max(bb - ab))
        best = None
        for j in (0, 1):
            sd = _side_distance(ab[j], bb[j], crossing[0].c[j])
            if sd is None:
                continue
            qual = min(_quality(Q, j, sd[0], Hb) for Q in crossing)
            if best is None or qual > best[1]:
                best = (j, qual, sd[1])
        if best is None or best[1] < beta:
            return False
        j2, _, side2 = best
    else:
        j2, side2 = 0, 1.0
    j3 = 1 - j2
    outer_breaks = []
    for Q in crossing:
        for edge in (ab[j2], bb[j2]):
            outer_breaks += Q.restrict(j2, edge).roots_1d()
    base_pts, base_w = [], []
    for lo3, hi3 in _pieces(ab[j3], bb[j3], outer_breaks):
        x3s, w3s = _gauss_on(lo3, hi3, n)
        for x3, w3 in zip(x3s, w3s):
            inner_breaks = []
            for Q in crossing:
                wq = Q.kappa - ((x3 - Q.c[j3]) / Q.s[j3]) ** 2
                if wq >= 0.0:
                    inner_breaks.append(Q.c[j2] + side2 * Q.s[j2] * np.sqrt(wq))
            for lo2, hi2 in _pieces(ab[j2], bb[j2], inner_breaks):
                x2s, w2s = _gauss_on(lo2, hi2, n)
                pts = np.zeros((n, 2))
                pts[:, j2] = x2s
                pts[:, j3] = x3
                base_pts.append(pts)
                base_w.append(w2s * w3)
    base = np.concatenate(base_pts)
    bw = np.concatenate(base_w)
    _column(q, e, side, a[e], b[e], base, bw, dims_base, n_t, rule)
    return True


def _box_rule(rule: Rule, q: Quadric, a, b, n, n_t, beta, depth, maxdepth):
    if q.box_min(a, b) >= 0.0:
        return
    if q.box_max(a, b) <= 0.0:
        _tensor_box(rule, a, b, n_t)
        return
    best = _best_direction(q, a, b, list(range(q.m)), beta)
    if best is not None:
        e, _, side = best
        if _integrate_plan(rule, q, a, b, e, side, n, n_t, beta):
            return
    if depth >= maxdepth:
        raise RuntimeError("cut-cell quadrature: subdivision depth exceeded")
    mid = 0.5 * (a + b)
    for corner in itertools.product((0, 1), repeat=q.m):
        ca = np.where(np.array(corner) == 0, a, mid)
        cb = np.where(np.array(corner) == 0, mid, b)
        _box_rule(rule, q, ca, cb, n, n_t, beta, depth + 1, maxdepth)


def cut_cell_rule(shape, box_lo, box_hi, n=16, n_t=None, beta=0.35, maxdepth=14):
    """Quadrature for T ∩ Omega and Gamma ∩ T with Omega = {q < 0} for one shape.

    Returns (vol_x, vol_w, surf_x, surf_w, surf_normal) in physical coordinates;
    the normal is the unit outward normal grad q / |grad q|.
    n: Gauss points per smooth piece in the base directions; n_t: Gauss points
    along the height direction (defaults to n).
    """
    q = Quadric(shape.center, shape.semi, 1.0)
    rule = Rule(q.m)
    a = np.asarray(box_lo, dtype=np.float64)
    b = np.asarray(box_hi, dtype=np.float64)
    _box_rule(rule, q, a, b, n, n if n_t is None else n_t, beta, 0, maxdepth)
    return rule.arrays()


# ---------------------------------------------------------------------------
# Unions of shapes.  Omega = union of the shapes; Gamma = the parts of the shape
# surfaces that lie outside every other shape.
#   * a box inside one shape is full; a box that no surface crosses is empty;
#   * a box crossed by exactly one surface (the other shapes disjoint from it)
#     uses the single-shape rule above;
#   * a box crossed by several surfaces is bisected up to `union_depth`; the
#     remaining leaves use columns along the last axis over an n^(d-1) Gauss
#     base grid, with the inside part of every column the exact union of the
#     per-shape intervals (roots of the quadratics) and boundary points at the
#     interval ends that lie inside the box.  This leaf rule is not exponentially
#     convergent (the union has kinks where two surfaces meet); it is a fixed,
#     deterministic rule.


def _union_leaf(rule: Rule, quads, a, b, n, n_t):
    d = len(a)
    e = d - 1
    base_dims = list(range(d - 1))
    xs, ws = zip(*[_gauss_on(a[j], b[j], n) for j in base_dims])
    grid = np.stack(np.meshgrid(*xs, indexing="ij"), axis=-1).reshape(-1, d - 1)
    wgt = np.ones(1)
    for j in range(d - 1):
        wgt = np.multiply.outer(wgt, ws[j])
    wgt = wgt.reshape(-1)
    xt, wt = gauss_legendre(n_t)
    for p in range(grid.shape[0]):
        xb = grid[p]
        ivs = []
        for qi, q in enumerate(quads):
            w = q.kappa - np.sum(((xb - q.c[:e]) / q.s[:e]) ** 2)
            if w <= 0.0:
                continue
            r = q.s[e] * np.sqrt(w)
            lo, hi = q.c[e] - r, q.c[e] + r
            lo_c, hi_c = max(lo, a[e]), min(hi, b[e])
            if hi_c > lo_c:
                ivs.append((lo_c, hi_c, qi if lo > a[e] else -1, qi if hi < b[e] else -1))
        if not ivs:
            continue
        ivs.sort(key=lambda v: (v[0], v[1]))
        merged = [list(ivs[0])]
        for lo, hi, olo, ohi in ivs[1:]:
            cur = merged[-1]
            if lo <= cur[1]:
                if hi > cur[1]:
                    cur[1], cur[3] = hi, ohi
            else:
                merged.append([lo, hi, olo, ohi])
        for lo, hi, olo, ohi in merged:
            pts = np.repeat(np.append(xb, 0.0)[None, :], n_t, axis=0)
            pts[:, e] = lo + (hi - lo) * xt
            rule.add_volume(pts, wgt[p] * (hi - lo) * wt)
            for t, owner in ((lo, olo), (hi, ohi)):
                if owner < 0:
                    continue
                q = quads[owner]
                sp = np.append(xb, t)
                g = q.grad(sp)
                gn = np.linalg.norm(g)
                rule.add_surface(sp[None, :], wgt[p] * gn / abs(g[e]), (g / gn)[None, :])


def _union_box(rule: Rule, quads, a, b, n, n_t, beta, depth, union_depth, maxdepth):
    if any(q.box_max(a, b) <= 0.0 for q in quads):
        _tensor_box(rule, a, b, n_t)
        return
    crossing = [q for q in quads if q.box_min(a, b) < 0.0 < q.box_max(a, b)]
    if not crossing:
        return
    if len(crossing) == 1:
        _box_rule(rule, crossing[0], a, b, n, n_t, beta, depth, maxdepth)
        return
    if depth >= union_depth:
        _union_leaf(rule, crossing, a, b, n, n_t)
        return
    mid = 0.5 * (a + b)
    for corner in itertools.product((0, 1), repeat=len(a)):
        ca = np.where(np.array(corner) == 0, a, mid)
        cb = np.where(np.array(corner) == 0, mid, b)
        _union_box(rule, quads, ca, cb, n, n_t, beta, depth + 1, union_depth, maxdepth)


def cut_cell_rule_union(shapes, box_lo, box_hi, n=14, n_t=None, beta=0.35, union_depth=4, maxdepth=14):
    """Quadrature of T ∩ (union of shapes) and of its boundary inside T (see above).
    With one shape this is exactly cut_cell_rule."""
    quads = [Quadric(s.center, s.semi, 1.0) for s in shapes]
    d = quads[0].m
    rule = Rule(d)
    a = np.asarray(box_lo, dtype=np.float64)
    b = np.asarray(box_hi, dtype=np.float64)
    _union_box(rule, quads, a, b, n, n if n_t is None else n_t, beta, 0, union_depth, maxdepth)
    return rule.arrays()
