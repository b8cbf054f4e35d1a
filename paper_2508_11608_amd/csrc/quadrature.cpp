// Cut-cell quadrature for the host set-up (paper, Section 3: substitute
// quadrature on cut cells, computed upfront on the CPU).
//
// Dimension reduction for an axis-aligned ellipsoid q(x) = sum ((x-c)/s)^2 - 1:
// a height direction e in which the box does not straddle the centre makes q
// monotone along every vertical line, so the inside part of each line is one
// interval whose end point t*(x') solves a quadratic.  The base integrand is
// analytic except on the traces of Gamma on the bottom and top faces (again
// ellipses), so the base is split there: at their roots in 2-D, and in 3-D by a
// second height direction inside the base with break points where the traces
// cross the base edges.  Boxes are bisected when no direction qualifies or when
// the square-root singularity of t* is close relative to the box size.
// The rule is emitted as columns (base point, weight, inside interval, boundary
// crossing), which the callers integrate in closed form or with Gauss points.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <vector>

#include "host.h"

namespace cmg {
namespace {

struct Quadric {  // sum_j ((x_j - c_j)/s_j)^2 - kappa over m dimensions
  int m;
  double c[kMaxDim], s[kMaxDim], kappa;

  double value(const double* x) const {
    double v = -kappa;
    for (int j = 0; j < m; ++j) {
      const double t = (x[j] - c[j]) / s[j];
      v += t * t;
    }
    return v;
  }
  double box_min(const double* a, const double* b) const {
    double v = -kappa;
    for (int j = 0; j < m; ++j) {
      const double d = std::max(std::max(a[j] - c[j], c[j] - b[j]), 0.0) / s[j];
      v += d * d;
    }
    return v;
  }
  double box_max(const double* a, const double* b) const {
    double v = -kappa;
    for (int j = 0; j < m; ++j) {
      const double d = std::max(std::fabs(a[j] - c[j]), std::fabs(b[j] - c[j])) / s[j];
      v += d * d;
    }
    return v;
  }
  bool crosses(const double* a, const double* b) const { return box_min(a, b) < 0.0 && box_max(a, b) > 0.0; }
  Quadric drop(int j, double val) const {  // fix x_j = val
    Quadric r;
    r.m = m - 1;
    int p = 0;
    for (int i = 0; i < m; ++i)
      if (i != j) { r.c[p] = c[i]; r.s[p] = s[i]; ++p; }
    const double t = (val - c[j]) / s[j];
    r.kappa = kappa - t * t;
    return r;
  }
};

// Distance of [a,b] from c when it does not straddle c; side +1 if above.
bool side_dist(double a, double b, double c, double& dist, double& side) {
  if (a >= c) { dist = a - c; side = 1.0; return true; }
  if (b <= c) { dist = c - b; side = -1.0; return true; }
  return false;
}

// Lower bound of the distance from the box to the branch point of t*(x'),
// relative to the box size H.
double quality(const Quadric& q, int e, double dist, double H) {
  double smin = 1e300;
  for (int j = 0; j < q.m; ++j)
    if (j != e) smin = std::min(smin, q.s[j]);
  if (q.m == 1) smin = q.s[e];
  const double u = dist / q.s[e];
  return u * u * smin / (2.0 * std::sqrt(std::max(q.kappa, 1e-300))) / H;
}

struct Gauss {
  std::vector<double> x, w;
  explicit Gauss(int n) : x(n), w(n) { gauss_legendre(n, x.data(), w.data()); }
};

void add_breaks(const Quadric& q1d, double lo, double hi, std::vector<double>& br) {
  if (q1d.kappa < 0.0) return;
  const double r = q1d.s[0] * std::sqrt(q1d.kappa);
  for (double t : {q1d.c[0] - r, q1d.c[0] + r})
    if (t > lo && t < hi) br.push_back(t);
}

std::vector<std::pair<double, double>> pieces(double lo, double hi, std::vector<double> br) {
  std::sort(br.begin(), br.end());
  std::vector<std::pair<double, double>> out;
  double prev = lo;
  for (double t : br) {
    if (t > prev) { out.push_back({prev, t}); prev = t; }
  }
  if (hi > prev) out.push_back({prev, hi});
  return out;
}

struct Ctx {
  int dim;
  Quadric q;
  int n, n_full;
  double beta;
  const Gauss* gn;
  const Gauss* gf;
  std::vector<Column>* out;
};

// Emit the column above base point xb (full coordinates, component e ignored).
void emit_column(const Ctx& C, int e, double side, double ae, double be, const double* xb, double wb) {
  const Quadric& q = C.q;
  Column col;
  col.e = e;
  for (int j = 0; j < kMaxDim; ++j) col.x[j] = (j < C.dim) ? xb[j] : 0.0;
  col.w = wb;
  double p[kMaxDim];
  for (int j = 0; j < C.dim; ++j) p[j] = xb[j];
  p[e] = ae;
  const double qa = q.value(p);
  p[e] = be;
  const double qb = q.value(p);
  double wq = q.kappa;
  for (int j = 0; j < C.dim; ++j)
    if (j != e) {
      const double t = (xb[j] - q.c[j]) / q.s[j];
      wq -= t * t;
    }
  const double ts = q.c[e] + side * q.s[e] * std::sqrt(std::max(wq, 0.0));
  const bool inA = qa < 0.0, inB = qb < 0.0;
  col.t0 = inA ? ae : ts;
  col.t1 = inB ? be : ts;
  if (!(inA || inB)) { col.t0 = 0.0; col.t1 = 0.0; }
  col.surf = inA != inB;
  col.ts = ts;
  col.sw = 0.0;
  if (col.surf) {
    p[e] = ts;
    double g[kMaxDim], gn = 0.0;
    for (int j = 0; j < C.dim; ++j) {
      g[j] = 2.0 * (p[j] - q.c[j]) / (q.s[j] * q.s[j]);
      gn += g[j] * g[j];
    }
    gn = std::sqrt(gn);
    col.sw = wb * gn / std::fabs(g[e]);
    for (int j = 0; j < C.dim; ++j) col.nrm[j] = g[j] / gn;
  }
  if (col.t1 > col.t0 || col.surf) C.out->push_back(col);
}

void full_box(const Ctx& C, const double* a, const double* b) {
  const int e = C.dim - 1;
  const Gauss& g = *C.gf;
  const int nf = C.n_full;
  double xb[kMaxDim] = {0, 0, 0};
  if (C.dim == 2) {
    for (int i = 0; i < nf; ++i) {
      xb[0] = a[0] + (b[0] - a[0]) * g.x[i];
      Column col{};
      col.e = e;
      col.x[0] = xb[0];
      col.w = (b[0] - a[0]) * g.w[i];
      col.t0 = a[e];
      col.t1 = b[e];
      col.surf = false;
      C.out->push_back(col);
    }
  } else {
    for (int j = 0; j < nf; ++j)
      for (int i = 0; i < nf; ++i) {
        Column col{};
        col.e = e;
        col.x[0] = a[0] + (b[0] - a[0]) * g.x[i];
        col.x[1] = a[1] + (b[1] - a[1]) * g.x[j];
        col.w = (b[0] - a[0]) * g.w[i] * (b[1] - a[1]) * g.w[j];
        col.t0 = a[e];
        col.t1 = b[e];
        col.surf = false;
        C.out->push_back(col);
      }
  }
}

bool plan(const Ctx& C, const double* a, const double* b, int e, double side) {
  const Quadric& q = C.q;
  const Gauss& g = *C.gn;
  const int n = C.n;
  int base[2], nb = 0;
  for (int j = 0; j < C.dim; ++j)
    if (j != e) base[nb++] = j;
  const Quadric Qa = q.drop(e, a[e]), Qb = q.drop(e, b[e]);
  double ab[2], bb[2];
  for (int j = 0; j < nb; ++j) { ab[j] = a[base[j]]; bb[j] = b[base[j]]; }
  double xb[kMaxDim] = {0, 0, 0};
  if (C.dim == 2) {
    std::vector<double> br;
    add_breaks(Qa, ab[0], bb[0], br);
    add_breaks(Qb, ab[0], bb[0], br);
    for (auto [lo, hi] : pieces(ab[0], bb[0], br))
      for (int i = 0; i < n; ++i) {
        xb[base[0]] = lo + (hi - lo) * g.x[i];
        emit_column(C, e, side, a[e], b[e], xb, (hi - lo) * g.w[i]);
      }
    return true;
  }
  // 3-D: base box in local coordinates (0, 1) -> global base[0], base[1].
  const Quadric* cross[2];
  int nc = 0;
  if (Qa.crosses(ab, bb)) cross[nc++] = &Qa;
  if (Qb.crosses(ab, bb)) cross[nc++] = &Qb;
  int j2 = 0;
  double side2 = 1.0;
  if (nc > 0) {
    const double Hb = std::max(bb[0] - ab[0], bb[1] - ab[1]);
    int best = -1;
    double bestq = -1.0, bestside = 1.0;
    for (int j = 0; j < 2; ++j) {
      double dist, sd;
      if (!side_dist(ab[j], bb[j], cross[0]->c[j], dist, sd)) continue;
      double qual = 1e300;
      for (int c = 0; c < nc; ++c) qual = std::min(qual, quality(*cross[c], j, dist, Hb));
      if (best < 0 || qual > bestq) { best = j; bestq = qual; bestside = sd; }
    }
    if (best < 0 || bestq < C.beta) return false;
    j2 = best;
    side2 = bestside;
  }
  const int j3 = 1 - j2;
  std::vector<double> obr;
  for (int c = 0; c < nc; ++c)
    for (double edge : {ab[j2], bb[j2]}) add_breaks(cross[c]->drop(j2, edge), ab[j3], bb[j3], obr);
  for (auto [lo3, hi3] : pieces(ab[j3], bb[j3], obr)) {
    for (int i3 = 0; i3 < n; ++i3) {
      const double x3 = lo3 + (hi3 - lo3) * g.x[i3];
      const double w3 = (hi3 - lo3) * g.w[i3];
      std::vector<double> ibr;
      for (int c = 0; c < nc; ++c) {
        const double t = (x3 - cross[c]->c[j3]) / cross[c]->s[j3];
        const double wq = cross[c]->kappa - t * t;
        if (wq >= 0.0) {
          const double r = cross[c]->c[j2] + side2 * cross[c]->s[j2] * std::sqrt(wq);
          if (r > ab[j2] && r < bb[j2]) ibr.push_back(r);
        }
      }
      for (auto [lo2, hi2] : pieces(ab[j2], bb[j2], ibr))
        for (int i2 = 0; i2 < n; ++i2) {
          xb[base[j2]] = lo2 + (hi2 - lo2) * g.x[i2];
          xb[base[j3]] = x3;
          emit_column(C, e, side, a[e], b[e], xb, (hi2 - lo2) * g.w[i2] * w3);
        }
    }
  }
  return true;
}

void box_rule(const Ctx& C, const double* a, const double* b, int depth) {
  const Quadric& q = C.q;
  if (q.box_min(a, b) >= 0.0) return;
  if (q.box_max(a, b) <= 0.0) { full_box(C, a, b); return; }
  double H = 0.0;
  for (int j = 0; j < C.dim; ++j) H = std::max(H, b[j] - a[j]);
  int best = -1;
  double bestq = -1.0, bestside = 1.0;
  for (int e = 0; e < C.dim; ++e) {
    double dist, sd;
    if (!side_dist(a[e], b[e], q.c[e], dist, sd)) continue;
    const double qual = quality(q, e, dist, H);
    if (best < 0 || qual > bestq) { best = e; bestq = qual; bestside = sd; }
  }
  if (best >= 0 && bestq >= C.beta && plan(C, a, b, best, bestside)) return;
  if (depth >= 14) throw std::runtime_error("cut-cell quadrature: subdivision depth exceeded");
  double mid[kMaxDim];
  for (int j = 0; j < C.dim; ++j) mid[j] = 0.5 * (a[j] + b[j]);
  for (int corner = 0; corner < (1 << C.dim); ++corner) {
    double ca[kMaxDim], cb[kMaxDim];
    for (int j = 0; j < C.dim; ++j) {
      const bool up = (corner >> j) & 1;
      ca[j] = up ? mid[j] : a[j];
      cb[j] = up ? b[j] : mid[j];
    }
    box_rule(C, ca, cb, depth + 1);
  }
}

// Union of shapes, box crossed by several surfaces at the maximal union depth:
// columns along the last axis over an n^(d-1) Gauss base grid; the inside part
// of a column is the exact union of the per-shape intervals, and every interval
// end inside the box is a boundary point of its shape.
void union_leaf(int dim, const std::vector<const Quadric*>& qs, const double* a, const double* b, const Gauss& g,
                int n, std::vector<Column>& out) {
  const int e = dim - 1;
  const int nb = dim == 2 ? n : n * n;
  struct Iv { double lo, hi; int olo, ohi; };
  std::vector<Iv> ivs;
  for (int p = 0; p < nb; ++p) {
    double xb[kMaxDim] = {0, 0, 0}, wb = 1.0;
    {
      int r = p;
      for (int j = 0; j < dim - 1; ++j) {
        const int i = r % n;
        r /= n;
        xb[j] = a[j] + (b[j] - a[j]) * g.x[i];
        wb *= (b[j] - a[j]) * g.w[i];
      }
    }
    ivs.clear();
    for (size_t qi = 0; qi < qs.size(); ++qi) {
      const Quadric& q = *qs[qi];
      double w = q.kappa;
      for (int j = 0; j < dim - 1; ++j) {
        const double t = (xb[j] - q.c[j]) / q.s[j];
        w -= t * t;
      }
      if (!(w > 0.0)) continue;
      const double r = q.s[e] * std::sqrt(w);
      const double lo = q.c[e] - r, hi = q.c[e] + r;
      const double lo_c = std::max(lo, a[e]), hi_c = std::min(hi, b[e]);
      if (hi_c > lo_c) ivs.push_back({lo_c, hi_c, lo > a[e] ? static_cast<int>(qi) : -1,
                                      hi < b[e] ? static_cast<int>(qi) : -1});
    }
    if (ivs.empty()) continue;
    std::sort(ivs.begin(), ivs.end(), [](const Iv& u, const Iv& v) {
      return u.lo < v.lo || (u.lo == v.lo && u.hi < v.hi);
    });
    std::vector<Iv> merged{ivs[0]};
    for (size_t i = 1; i < ivs.size(); ++i) {
      Iv& cur = merged.back();
      if (ivs[i].lo <= cur.hi) {
        if (ivs[i].hi > cur.hi) { cur.hi = ivs[i].hi; cur.ohi = ivs[i].ohi; }
      } else {
        merged.push_back(ivs[i]);
      }
    }
    for (const Iv& iv : merged) {
      Column col{};
      col.e = e;
      for (int j = 0; j < dim - 1; ++j) col.x[j] = xb[j];
      col.w = wb;
      col.t0 = iv.lo;
      col.t1 = iv.hi;
      col.surf = false;
      out.push_back(col);
      for (int end = 0; end < 2; ++end) {
        const int owner = end ? iv.ohi : iv.olo;
        if (owner < 0) continue;
        const Quadric& q = *qs[owner];
        Column sc{};
        sc.e = e;
        for (int j = 0; j < dim - 1; ++j) sc.x[j] = xb[j];
        sc.w = wb;
        sc.t0 = sc.t1 = 0.0;
        sc.surf = true;
        sc.ts = end ? iv.hi : iv.lo;
        double pt[kMaxDim], gq[kMaxDim], gn = 0.0;
        for (int j = 0; j < dim; ++j) pt[j] = j == e ? sc.ts : xb[j];
        for (int j = 0; j < dim; ++j) {
          gq[j] = 2.0 * (pt[j] - q.c[j]) / (q.s[j] * q.s[j]);
          gn += gq[j] * gq[j];
        }
        gn = std::sqrt(gn);
        sc.sw = wb * gn / std::fabs(gq[e]);
        for (int j = 0; j < dim; ++j) sc.nrm[j] = gq[j] / gn;
        out.push_back(sc);
      }
    }
  }
}

void union_box(const Ctx& base, const std::vector<Quadric>& qs, const double* a, const double* b, int depth,
               int union_depth) {
  const int dim = base.dim;
  for (const Quadric& q : qs)
    if (q.box_max(a, b) <= 0.0) { full_box(base, a, b); return; }
  std::vector<const Quadric*> crossing;
  for (const Quadric& q : qs)
    if (q.box_min(a, b) < 0.0 && q.box_max(a, b) > 0.0) crossing.push_back(&q);
  if (crossing.empty()) return;
  if (crossing.size() == 1) {
    Ctx C = base;
    C.q = *crossing[0];
    box_rule(C, a, b, depth);
    return;
  }
  if (depth >= union_depth) {
    union_leaf(dim, crossing, a, b, *base.gn, base.n, *base.out);
    return;
  }
  double mid[kMaxDim];
  for (int j = 0; j < dim; ++j) mid[j] = 0.5 * (a[j] + b[j]);
  for (int corner = 0; corner < (1 << dim); ++corner) {
    double ca[kMaxDim], cb[kMaxDim];
    for (int j = 0; j < dim; ++j) {
      const bool up = (corner >> j) & 1;
      ca[j] = up ? mid[j] : a[j];
      cb[j] = up ? b[j] : mid[j];
    }
    union_box(base, qs, ca, cb, depth + 1, union_depth);
  }
}

}  // namespace

void cut_columns_union(int dim, const std::vector<Shape>& shapes, const double* a, const double* b, int n,
                       int n_full, double beta, int union_depth, std::vector<Column>& out) {
  std::vector<Quadric> qs(shapes.size());
  for (size_t i = 0; i < shapes.size(); ++i) {
    qs[i].m = dim;
    for (int j = 0; j < dim; ++j) { qs[i].c[j] = shapes[i].c[j]; qs[i].s[j] = shapes[i].s[j]; }
    qs[i].kappa = 1.0;
  }
  Ctx C;
  C.dim = dim;
  C.q = qs[0];
  C.n = n;
  C.n_full = n_full;
  C.beta = beta;
  Gauss gn(n), gf(n_full);
  C.gn = &gn;
  C.gf = &gf;
  C.out = &out;
  union_box(C, qs, a, b, 0, union_depth);
}

void cut_columns(int dim, const Shape& sh, const double* a, const double* b, int n, int n_full,
                 double beta, std::vector<Column>& out) {
  Ctx C;
  C.dim = dim;
  C.q.m = dim;
  for (int j = 0; j < dim; ++j) { C.q.c[j] = sh.c[j]; C.q.s[j] = sh.s[j]; }
  C.q.kappa = 1.0;
  C.n = n;
  C.n_full = n_full;
  C.beta = beta;
  Gauss gn(n), gf(n_full);
  C.gn = &gn;
  C.gf = &gf;
  C.out = &out;
  box_rule(C, a, b, 0);
}

}  // namespace cmg
