// Host set-up of the level hierarchy (paper, Sections 2 and 3).
//
//  * Levels l = 0..L-1 of a Cartesian background mesh, N_l = N_0 2^l cells per
//    direction; cells are active when they meet Omega and cut when they are
//    active but not inside one shape (strict inequalities); DoFs are the nodes
//    of the (kN+1)^d Gauss-Lobatto lattice in the closure of an active cell.
//  * Element matrices: uncut cells by the tensor formula K = h^{d-2} sum_j
//    M x..x K(j) x..x M; cut cells from volume and surface moments of the cut
//    rule in a shifted Legendre basis (volume term, Nitsche terms, penalty
//    gamma_D/h).
//  * Ghost faces: faces between two active cells with at least one cut; the
//    face matrix is the same for every face of one direction on a level.
//  * Vertex patches around every vertex of an active cell, coloured by the
//    parity of the vertex index; interior patches (Cartesian local matrix) use
//    fast diagonalisation, all others a dense inverse of the principal
//    submatrix of A_l, computed in FP64 by Cholesky.
//  * The exact coarse solver is a dense inverse of A_0.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <stdexcept>

#include "host.h"

namespace cmg {
namespace {

int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// Shifted Legendre polynomials L_p(t) = P_p(2t - 1) on [0,1] (values up to p = n-1).
void legendre_values(double t, int n, double* v) {
  const double s = 2.0 * t - 1.0;
  v[0] = 1.0;
  if (n > 1) v[1] = s;
  for (int p = 2; p < n; ++p) v[p] = ((2.0 * p - 1.0) * s * v[p - 1] - (p - 1.0) * v[p - 2]) / p;
}

// int_{t0}^{t1} L_p(t) dt for p < n, from the antiderivative (P_{p+1} - P_{p-1})/(2p+1).
void legendre_integrals(double t0, double t1, int n, double* out) {
  double v0[2 * kMaxDeg + 3], v1[2 * kMaxDeg + 3];
  legendre_values(t0, n + 1, v0);
  legendre_values(t1, n + 1, v1);
  const double s0 = 2.0 * t0 - 1.0, s1 = 2.0 * t1 - 1.0;
  out[0] = 0.5 * (s1 - s0);
  for (int p = 1; p < n; ++p) out[p] = 0.5 * ((v1[p + 1] - v1[p - 1]) - (v0[p + 1] - v0[p - 1])) / (2.0 * p + 1.0);
}

// Legendre coefficients of products of two 1-D basis polynomials or derivatives:
// psi_a psi_b = sum_p c[0][a][b][p] L_p, and likewise psi_a' psi_b' (kind 1) and
// psi_a' psi_b (kind 2).  The Legendre basis keeps the moment sums well
// conditioned for k = 3.
struct PairPoly {
  int k;
  double c[3][kMaxDeg + 1][kMaxDeg + 1][2 * kMaxDeg + 1];
};

PairPoly make_pairpoly(const Basis1D& B) {
  PairPoly P;
  P.k = B.k;
  std::memset(P.c, 0, sizeof P.c);
  const int k = B.k, na = 2 * k + 1;
  const int ng = 2 * k + 2;  // exact for degree 4k + 1
  double gx[2 * kMaxDeg + 2], gw[2 * kMaxDeg + 2];
  gauss_legendre(ng, gx, gw);
  for (int q = 0; q < ng; ++q) {
    double L[2 * kMaxDeg + 1];
    legendre_values(gx[q], na, L);
    for (int a = 0; a <= k; ++a)
      for (int b = 0; b <= k; ++b) {
        const double f0 = B.eval(a, gx[q]) * B.eval(b, gx[q]);
        const double f1 = B.eval(a, gx[q], 1) * B.eval(b, gx[q], 1);
        const double f2 = B.eval(a, gx[q], 1) * B.eval(b, gx[q]);
        for (int p = 0; p < na; ++p) {
          const double wl = gw[q] * L[p] * (2.0 * p + 1.0);
          P.c[0][a][b][p] += wl * f0;
          P.c[1][a][b][p] += wl * f1;
          P.c[2][a][b][p] += wl * f2;
        }
      }
  }
  return P;
}

// E[a,b] += scale * sum_alpha prod_i F_i[a_i][b_i][alpha_i] mom[alpha], with F_i
// chosen per dimension (kind[i], transposed[i]) and alpha in [0, 2k]^d (x fastest).
void contract(int d, int k, const PairPoly& P, const int* kind, const bool* transp, const double* mom,
              double scale, double* E) {
  const int n1 = k + 1, na = 2 * k + 1, nl = ipow(n1, d);
  auto F = [&](int i, int a, int b, int p) {
    return transp[i] ? P.c[kind[i]][b][a][p] : P.c[kind[i]][a][b][p];
  };
  if (d == 2) {
    // T[a0,b0][al1] = sum_al0 F0 mom[al0 + na al1]
    std::vector<double> T(n1 * n1 * na);
    for (int a0 = 0; a0 < n1; ++a0)
      for (int b0 = 0; b0 < n1; ++b0)
        for (int l1 = 0; l1 < na; ++l1) {
          double s = 0;
          for (int l0 = 0; l0 < na; ++l0) s += F(0, a0, b0, l0) * mom[l0 + na * l1];
          T[(a0 * n1 + b0) * na + l1] = s;
        }
    for (int a1 = 0; a1 < n1; ++a1)
      for (int b1 = 0; b1 < n1; ++b1)
        for (int a0 = 0; a0 < n1; ++a0)
          for (int b0 = 0; b0 < n1; ++b0) {
            double s = 0;
            for (int l1 = 0; l1 < na; ++l1) s += F(1, a1, b1, l1) * T[(a0 * n1 + b0) * na + l1];
            E[(a0 + n1 * a1) * nl + (b0 + n1 * b1)] += scale * s;
          }
    return;
  }
  std::vector<double> T1(n1 * n1 * na * na), T2(n1 * n1 * n1 * n1 * na);
  for (int a0 = 0; a0 < n1; ++a0)
    for (int b0 = 0; b0 < n1; ++b0)
      for (int l2 = 0; l2 < na; ++l2)
        for (int l1 = 0; l1 < na; ++l1) {
          double s = 0;
          for (int l0 = 0; l0 < na; ++l0) s += F(0, a0, b0, l0) * mom[l0 + na * (l1 + na * l2)];
          T1[((a0 * n1 + b0) * na + l1) * na + l2] = s;
        }
  for (int a0 = 0; a0 < n1; ++a0)
    for (int b0 = 0; b0 < n1; ++b0)
      for (int a1 = 0; a1 < n1; ++a1)
        for (int b1 = 0; b1 < n1; ++b1)
          for (int l2 = 0; l2 < na; ++l2) {
            double s = 0;
            for (int l1 = 0; l1 < na; ++l1) s += F(1, a1, b1, l1) * T1[((a0 * n1 + b0) * na + l1) * na + l2];
            T2[(((a0 * n1 + b0) * n1 + a1) * n1 + b1) * na + l2] = s;
          }
  for (int a2 = 0; a2 < n1; ++a2)
    for (int b2 = 0; b2 < n1; ++b2)
      for (int a1 = 0; a1 < n1; ++a1)
        for (int b1 = 0; b1 < n1; ++b1)
          for (int a0 = 0; a0 < n1; ++a0)
            for (int b0 = 0; b0 < n1; ++b0) {
              double s = 0;
              for (int l2 = 0; l2 < na; ++l2)
                s += F(2, a2, b2, l2) * T2[(((a0 * n1 + b0) * n1 + a1) * n1 + b1) * na + l2];
              E[(a0 + n1 * (a1 + n1 * a2)) * nl + (b0 + n1 * (b1 + n1 * b2))] += scale * s;
            }
}

// Reference 1-D mass and stiffness on [0,1] (exact Gauss rule).
void ref_1d(const Basis1D& B, double* M, double* K) {
  const int k = B.k, n1 = k + 1;
  double x[kMaxDeg + 2], w[kMaxDeg + 2];
  gauss_legendre(k + 1, x, w);
  for (int a = 0; a < n1; ++a)
    for (int b = 0; b < n1; ++b) {
      double m = 0, s = 0;
      for (int p = 0; p <= k; ++p) {
        m += w[p] * B.eval(a, x[p]) * B.eval(b, x[p]);
        s += w[p] * B.eval(a, x[p], 1) * B.eval(b, x[p], 1);
      }
      M[a * n1 + b] = m;
      K[a * n1 + b] = s;
    }
}

bool shape_active(const Config& c, const double* lo, const double* hi) {
  for (const Shape& s : c.shapes) {
    double v = -1.0;
    for (int j = 0; j < c.dim; ++j) {
      const double d = std::max(std::max(lo[j] - s.c[j], s.c[j] - hi[j]), 0.0) / s.s[j];
      v += d * d;
    }
    if (v < 0.0) return true;
  }
  return false;
}

bool shape_inside(const Config& c, const double* lo, const double* hi) {
  for (const Shape& s : c.shapes) {
    double v = -1.0;
    for (int j = 0; j < c.dim; ++j) {
      const double d = std::max(std::fabs(lo[j] - s.c[j]), std::fabs(hi[j] - s.c[j])) / s.s[j];
      v += d * d;
    }
    if (v < 0.0) return true;
  }
  return false;
}

struct LevelGeom {
  int d, k, N, nn;
  int64_t cell(const int* c) const { return d == 2 ? c[0] + (int64_t)N * c[1] : c[0] + (int64_t)N * (c[1] + (int64_t)N * c[2]); }
  int64_t node(const int* I) const { return d == 2 ? I[0] + (int64_t)nn * I[1] : I[0] + (int64_t)nn * (I[1] + (int64_t)nn * I[2]); }
  void cell_of(int64_t lin, int* c) const {
    for (int j = 0; j < d; ++j) { c[j] = lin % N; lin /= N; }
  }
};

void classify(const Config& cfg, int N, HostLevel& L, const HostLevel* parent, std::string& err) {
  const int d = cfg.dim, k = cfg.k;
  L.N = N;
  L.nn = k * N + 1;
  L.h = (cfg.hi - cfg.lo) / N;
  L.n_cells = ipow(N, d);
  L.n_nodes = ipow(L.nn, d);
  L.cell_flags.assign(L.n_cells, 0);
  LevelGeom G{d, k, N, L.nn};
  for (int64_t c = 0; c < L.n_cells; ++c) {
    int ci[kMaxDim];
    G.cell_of(c, ci);
    double lo[kMaxDim], hi[kMaxDim];
    for (int j = 0; j < d; ++j) {
      lo[j] = cfg.lo + ci[j] * L.h;
      hi[j] = cfg.lo + (ci[j] + 1) * L.h;
    }
    if (shape_active(cfg, lo, hi)) {
      L.cell_flags[c] = kActive | (shape_inside(cfg, lo, hi) ? 0 : kCut);
      if (parent) {
        int pc[kMaxDim];
        for (int j = 0; j < d; ++j) pc[j] = ci[j] / 2;
        LevelGeom PG{d, k, N / 2, parent->nn};
        if (!(parent->cell_flags[PG.cell(pc)] & kActive)) err = "EGEOM: active cell with inactive parent";
      }
    }
  }
  // DoFs: nodes in the closure of an active cell, canonical (ascending lattice) order.
  std::vector<uint8_t> na(L.n_nodes, 0);
  const int n1 = k + 1;
  for (int64_t c = 0; c < L.n_cells; ++c) {
    if (!(L.cell_flags[c] & kActive)) continue;
    int ci[kMaxDim];
    G.cell_of(c, ci);
    for (int loc = 0; loc < ipow(n1, d); ++loc) {
      int I[kMaxDim];
      int r = loc;
      for (int j = 0; j < d; ++j) { I[j] = k * ci[j] + r % n1; r /= n1; }
      na[G.node(I)] = 1;
    }
  }
  L.node_dof.assign(L.n_nodes, -1);
  L.dof_node.clear();
  for (int64_t n = 0; n < L.n_nodes; ++n)
    if (na[n]) {
      L.node_dof[n] = static_cast<int32_t>(L.dof_node.size());
      L.dof_node.push_back(static_cast<int32_t>(n));
    }
  L.n_dofs = L.dof_node.size();
  // Ghost faces.
  L.ghost_mask.assign(L.n_cells, 0);
  for (int64_t c = 0; c < L.n_cells; ++c) {
    if (!(L.cell_flags[c] & kActive)) continue;
    int ci[kMaxDim];
    G.cell_of(c, ci);
    for (int dir = 0; dir < d; ++dir) {
      if (ci[dir] + 1 >= N) continue;
      int nb[kMaxDim];
      std::memcpy(nb, ci, sizeof nb);
      nb[dir] += 1;
      const int64_t cn = G.cell(nb);
      if ((L.cell_flags[cn] & kActive) && ((L.cell_flags[c] | L.cell_flags[cn]) & kCut)) {
        L.ghost_mask[c] |= 1 << (2 * dir + 1);
        L.ghost_mask[cn] |= 1 << (2 * dir + 0);
      }
    }
  }
  // Ghost face list (lower cell, direction) and, per cell with ghost faces, the
  // ids of its 2d faces (-1 where the face is not a ghost face).
  L.cell_gid.assign(L.n_cells, -1);
  L.cell_faces.clear();
  int32_t ng = 0;
  for (int64_t c = 0; c < L.n_cells; ++c)
    if (L.ghost_mask[c]) {
      L.cell_gid[c] = ng++;
      L.cell_faces.insert(L.cell_faces.end(), 2 * d, -1);
    }
  L.face_lower.clear();
  L.face_dir.clear();
  for (int64_t c = 0; c < L.n_cells; ++c) {
    if (!L.ghost_mask[c]) continue;
    int ci[kMaxDim];
    G.cell_of(c, ci);
    for (int dir = 0; dir < d; ++dir) {
      if (!(L.ghost_mask[c] & (1 << (2 * dir + 1)))) continue;
      int nb[kMaxDim];
      std::memcpy(nb, ci, sizeof nb);
      nb[dir] += 1;
      const int32_t fid = static_cast<int32_t>(L.face_lower.size());
      L.face_lower.push_back(static_cast<int32_t>(c));
      L.face_dir.push_back(static_cast<uint8_t>(dir));
      L.cell_faces[static_cast<size_t>(L.cell_gid[c]) * 2 * d + 2 * dir + 1] = fid;
      L.cell_faces[static_cast<size_t>(L.cell_gid[G.cell(nb)]) * 2 * d + 2 * dir] = fid;
    }
  }
  // Tiles of B^d cells for the operator kernel; a tile owns the nodes
  // [B k t, B k (t+1)) per direction (the last tile also the upper boundary) and is
  // listed when it owns an active node.
  const int B = (d == 3 && k == 3) ? 2 : 4;
  const int NTd = (N + B - 1) / B;
  std::vector<uint8_t> tile_used(static_cast<size_t>(ipow(NTd, d)), 0);
  for (int32_t node : L.dof_node) {
    int64_t r = node, t = 0, stride = 1;
    for (int j = 0; j < d; ++j) {
      const int I = static_cast<int>(r % L.nn);
      r /= L.nn;
      t += std::min(I / (B * k), NTd - 1) * stride;
      stride *= NTd;
    }
    tile_used[t] = 1;
  }
  L.tiles.clear();
  for (size_t t = 0; t < tile_used.size(); ++t)
    if (tile_used[t]) L.tiles.push_back(static_cast<int32_t>(t));
}

// Dense assembly of A restricted to a node set (map node -> position), from the
// given cells and from the ghost faces owned by them.
struct Assembler {
  const Config& cfg;
  const HostLevel& L;
  const std::vector<double>& K;        // uncut cell matrix
  const std::vector<double>* G;        // ghost matrix per direction
  int d, k, n1, nl;
  LevelGeom geo;

  void cell_nodes(const int* ci, int64_t* nodes) const {
    for (int loc = 0; loc < nl; ++loc) {
      int I[kMaxDim];
      int r = loc;
      for (int j = 0; j < d; ++j) { I[j] = k * ci[j] + r % n1; r /= n1; }
      nodes[loc] = geo.node(I);
    }
  }

  template <class Map>
  void add_cell(const int* ci, const Map& pos, double* A, int n) const {
    const int64_t c = geo.cell(ci);
    const uint8_t f = L.cell_flags[c];
    if (!(f & kActive)) return;
    const double* E = (f & kCut) ? &L.cut_mats[static_cast<size_t>(L.cut_id[c]) * nl * nl] : K.data();
    int64_t nodes[64 * 2];
    cell_nodes(ci, nodes);
    int p[64];
    for (int a = 0; a < nl; ++a) p[a] = pos(nodes[a]);
    for (int a = 0; a < nl; ++a) {
      if (p[a] < 0) continue;
      for (int b = 0; b < nl; ++b)
        if (p[b] >= 0) A[static_cast<size_t>(p[a]) * n + p[b]] += E[a * nl + b];
    }
  }

  template <class Map>
  void add_face(const int* lower, int dir, const Map& pos, double* A, int n) const {
    int upper[kMaxDim];
    std::memcpy(upper, lower, sizeof upper);
    upper[dir] += 1;
    int64_t nodes[128];
    cell_nodes(lower, nodes);
    cell_nodes(upper, nodes + nl);
    int p[128];
    for (int a = 0; a < 2 * nl; ++a) p[a] = pos(nodes[a]);
    const double* Gd = G[dir].data();
    for (int a = 0; a < 2 * nl; ++a) {
      if (p[a] < 0) continue;
      for (int b = 0; b < 2 * nl; ++b)
        if (p[b] >= 0) A[static_cast<size_t>(p[a]) * n + p[b]] += Gd[a * 2 * nl + b];
    }
  }
};

}  // namespace

void uncut_cell_matrix(const Config& cfg, const Basis1D& B, double h, std::vector<double>& K) {
  const int d = cfg.dim, k = cfg.k, n1 = k + 1, nl = ipow(n1, d);
  double M1[16], K1[16];
  ref_1d(B, M1, K1);
  K.assign(static_cast<size_t>(nl) * nl, 0.0);
  const double sc = std::pow(h, d - 2);
  for (int a = 0; a < nl; ++a)
    for (int b = 0; b < nl; ++b) {
      int ai[kMaxDim], bi[kMaxDim];
      for (int j = 0, ra = a, rb = b; j < d; ++j) { ai[j] = ra % n1; ra /= n1; bi[j] = rb % n1; rb /= n1; }
      double s = 0;
      for (int j = 0; j < d; ++j) {
        double t = 1;
        for (int i = 0; i < d; ++i) t *= (i == j ? K1 : M1)[ai[i] * n1 + bi[i]];
        s += t;
      }
      K[a * nl + b] = sc * s;
    }
}

void cut_cell_matrix(const Config& cfg, const Basis1D& B, double h, const double* lo, std::vector<double>& E) {
  const int d = cfg.dim, k = cfg.k, na = 2 * k + 1, nl = ipow(k + 1, d), nm = ipow(na, d);
  std::vector<Column> cols;
  double hi[kMaxDim];
  for (int j = 0; j < d; ++j) hi[j] = lo[j] + h;
  cut_columns_union(d, cfg.shapes, lo, hi, cfg.quad_n, k + 1, cfg.quad_beta, cfg.union_depth, cols);
  // Legendre moments in local coordinates xi = (x - lo)/h: volume, surface,
  // surface times n_j.
  std::vector<double> mv(nm, 0.0), ms(nm, 0.0), mn(static_cast<size_t>(d) * nm, 0.0);
  for (const Column& c : cols) {
    double pw[kMaxDim][2 * kMaxDeg + 2];
    for (int j = 0; j < d; ++j) {
      if (j == c.e) continue;
      legendre_values((c.x[j] - lo[j]) / h, na, pw[j]);
    }
    if (c.t1 > c.t0) {
      // closed-form integral of L_p(xi_e) over the inside interval, in physical measure
      legendre_integrals((c.t0 - lo[c.e]) / h, (c.t1 - lo[c.e]) / h, na, pw[c.e]);
      for (int p = 0; p < na; ++p) pw[c.e][p] *= h;
      for (int a = 0; a < nm; ++a) {
        double v = c.w;
        for (int j = 0, r = a; j < d; ++j) { v *= pw[j][r % na]; r /= na; }
        mv[a] += v;
      }
    }
    if (c.surf) {
      legendre_values((c.ts - lo[c.e]) / h, na, pw[c.e]);
      for (int a = 0; a < nm; ++a) {
        double v = c.sw;
        for (int j = 0, r = a; j < d; ++j) { v *= pw[j][r % na]; r /= na; }
        ms[a] += v;
        for (int j = 0; j < d; ++j) mn[static_cast<size_t>(j) * nm + a] += v * c.nrm[j];
      }
    }
  }
  const PairPoly P = make_pairpoly(B);
  E.assign(static_cast<size_t>(nl) * nl, 0.0);
  int kind[kMaxDim];
  bool tr[kMaxDim] = {false, false, false};
  // (grad u, grad v): h^{-2} per direction with psi'psi' in that direction.
  for (int j = 0; j < d; ++j) {
    for (int i = 0; i < d; ++i) kind[i] = (i == j) ? 1 : 0;
    contract(d, k, P, kind, tr, mv.data(), 1.0 / (h * h), E.data());
  }
  // -(d_n u, v) - (u, d_n v): h^{-1} n_j psi' psi in direction j, both orders.
  for (int j = 0; j < d; ++j) {
    for (int i = 0; i < d; ++i) kind[i] = (i == j) ? 2 : 0;
    bool t0[kMaxDim] = {false, false, false}, t1[kMaxDim] = {false, false, false};
    t1[j] = true;
    contract(d, k, P, kind, t0, &mn[static_cast<size_t>(j) * nm], -1.0 / h, E.data());
    contract(d, k, P, kind, t1, &mn[static_cast<size_t>(j) * nm], -1.0 / h, E.data());
  }
  // (gamma_D / h)(u, v)_Gamma
  for (int i = 0; i < d; ++i) kind[i] = 0;
  contract(d, k, P, kind, tr, ms.data(), cfg.gamma_D / h, E.data());
}

void ghost_face_matrix(const Config& cfg, const Basis1D& B, double h, int dir, std::vector<double>& G) {
  // Acts on [dofs(lower cell); dofs(upper cell)]; the jump of the m-th normal
  // derivative is (trace of the lower cell at xi=1) - (trace of the upper at xi=0).
  const int d = cfg.dim, k = cfg.k, n1 = k + 1, nl = ipow(n1, d);
  double M1[16], K1[16];
  ref_1d(B, M1, K1);
  G.assign(static_cast<size_t>(4) * nl * nl, 0.0);
  for (int m = 1; m <= k; ++m) {
    const int expo = cfg.ghost_exp_mode == 0 ? 2 * m - 1 : 2 * m + 1;
    double fact = 1.0;
    for (int i = 2; i <= m; ++i) fact *= i;
    const double c = cfg.gamma(m) * std::pow(h, expo - 2 * m + d - 1) / (fact * fact);
    for (int sa = 0; sa < 2; ++sa)
      for (int a = 0; a < nl; ++a)
        for (int sb = 0; sb < 2; ++sb)
          for (int b = 0; b < nl; ++b) {
            int ai[kMaxDim], bi[kMaxDim];
            for (int j = 0, ra = a, rb = b; j < d; ++j) { ai[j] = ra % n1; ra /= n1; bi[j] = rb % n1; rb /= n1; }
            const double ja = sa == 0 ? B.eval(ai[dir], 1.0, m) : -B.eval(ai[dir], 0.0, m);
            const double jb = sb == 0 ? B.eval(bi[dir], 1.0, m) : -B.eval(bi[dir], 0.0, m);
            double t = c * ja * jb;
            for (int j = 0; j < d; ++j)
              if (j != dir) t *= M1[ai[j] * n1 + bi[j]];
            G[static_cast<size_t>(sa * nl + a) * 2 * nl + sb * nl + b] += t;
          }
  }
}

void cut_step_sets(HostLevel& L, int d, int k);

std::string build_hierarchy(const Config& cfg, Hierarchy& H, bool numeric) {
  if (cfg.dim < 2 || cfg.dim > 3 || cfg.k < 1 || cfg.k > kMaxDeg || cfg.n_levels < 1 || cfg.coarse_cells < 1)
    return "EINVAL: unsupported dimension, degree or level count";
  if (cfg.shapes.empty()) return "EINVAL: no shapes";
  H.cfg = cfg;
  H.basis = make_basis(cfg.k);
  const int d = cfg.dim, k = cfg.k, n1 = k + 1, nl = ipow(n1, d);
  H.levels.assign(cfg.n_levels, HostLevel());
  H.tables.assign(cfg.n_levels, LevelTables());
  std::string err;
  for (int l = 0; l < cfg.n_levels; ++l) {
    classify(cfg, cfg.coarse_cells << l, H.levels[l], l ? &H.levels[l - 1] : nullptr, err);
    if (!err.empty()) return err;
  }
  if (H.levels[0].n_dofs == 0) return "EGEOM: no active cells on the coarsest level";
  double M1[16], K1[16];
  ref_1d(H.basis, M1, K1);
  try {
    for (int l = 0; l < cfg.n_levels; ++l) {
      HostLevel& L = H.levels[l];
      LevelTables& T = H.tables[l];
      LevelGeom geo{d, k, L.N, L.nn};
      // cut-cell element matrices
      L.cut_id.assign(L.n_cells, -1);
      std::vector<int64_t> cuts;
      for (int64_t c = 0; c < L.n_cells; ++c)
        if (L.cell_flags[c] & kCut) { L.cut_id[c] = static_cast<int32_t>(cuts.size()); cuts.push_back(c); }
      L.n_cut = static_cast<int>(cuts.size());
      L.cut_mats.assign(numeric ? static_cast<size_t>(L.n_cut) * nl * nl : 0, 0.0);
      std::string qerr;
      if (!numeric) cuts.clear();  // counts only: no cut-cell quadrature
#pragma omp parallel for schedule(dynamic, 4)
      for (int i = 0; i < static_cast<int>(cuts.size()); ++i) {
        int ci[kMaxDim];
        geo.cell_of(cuts[i], ci);
        double lo[kMaxDim];
        for (int j = 0; j < d; ++j) lo[j] = cfg.lo + ci[j] * L.h;
        std::vector<double> E;
        try {
          cut_cell_matrix(cfg, H.basis, L.h, lo, E);
        } catch (const std::exception& ex) {
#pragma omp critical
          qerr = std::string("EINVAL: ") + ex.what();
          continue;
        }
        std::copy(E.begin(), E.end(), L.cut_mats.begin() + static_cast<size_t>(i) * nl * nl);
      }
      if (!qerr.empty()) return qerr;
      // kernel tables
      uncut_cell_matrix(cfg, H.basis, L.h, T.kcell);
      T.mhat.assign(M1, M1 + n1 * n1);
      T.d0.assign(k * n1, 0.0);
      T.d1.assign(k * n1, 0.0);
      T.gcoef.assign(k, 0.0);
      for (int m = 1; m <= k; ++m) {
        for (int a = 0; a <= k; ++a) {
          T.d0[(m - 1) * n1 + a] = H.basis.eval(a, 0.0, m);
          T.d1[(m - 1) * n1 + a] = H.basis.eval(a, 1.0, m);
        }
        const int expo = cfg.ghost_exp_mode == 0 ? 2 * m - 1 : 2 * m + 1;
        double fact = 1.0;
        for (int i = 2; i <= m; ++i) fact *= i;
        T.gcoef[m - 1] = cfg.gamma(m) * std::pow(L.h, expo - 2 * m + d - 1) / (fact * fact);
      }
      // fast diagonalisation of the Cartesian patch Laplacian: 1-D patch matrices on
      // two cells, internal nodes 1..2k-1
      const int np1 = 2 * k - 1, nb1 = 2 * k + 1;
      std::vector<double> Kp(nb1 * nb1, 0.0), Mp(nb1 * nb1, 0.0);
      for (int c = 0; c < 2; ++c)
        for (int a = 0; a <= k; ++a)
          for (int b = 0; b <= k; ++b) {
            Kp[(k * c + a) * nb1 + k * c + b] += K1[a * n1 + b];
            Mp[(k * c + a) * nb1 + k * c + b] += M1[a * n1 + b];
          }
      std::vector<double> Ki(np1 * np1), Mi(np1 * np1), S(np1 * np1), lam(np1);
      for (int i = 0; i < np1; ++i)
        for (int j = 0; j < np1; ++j) {
          Ki[i * np1 + j] = Kp[(i + 1) * nb1 + j + 1];
          Mi[i * np1 + j] = Mp[(i + 1) * nb1 + j + 1];
        }
      if (!gen_eig(np1, Ki.data(), Mi.data(), S.data(), lam.data())) return "ENOTSPD: 1-D patch mass";
      T.fd_s = S;
      const int npd = ipow(np1, d);
      T.fd_dinv.assign(npd, 0.0);
      const double hs = std::pow(L.h, 2 - d);
      for (int i = 0; i < npd; ++i) {
        double s = 0;
        for (int j = 0, r = i; j < d; ++j) { s += lam[r % np1]; r /= np1; }
        T.fd_dinv[i] = hs / s;
      }
      // prolongation weights: fine node q in [0, 2k] of a coarse cell, coarse basis b
      T.p1d.assign((2 * k + 1) * n1, 0.0);
      for (int q = 0; q <= 2 * k; ++q) {
        const int f = q / k, a = q % k;
        const double eta = q == 2 * k ? 1.0 : 0.5 * (f + H.basis.node[a]);
        for (int b = 0; b <= k; ++b) T.p1d[q * n1 + b] = H.basis.eval(b, eta);
      }
      // reference 1-D stiffness times h^(d-2): the uncut cell stiffness is the
      // sum over directions a of the tensor products with this factor along a
      // and the reference 1-D mass along the others
      T.k1s.assign(n1 * n1, 0.0);
      for (int i = 0; i < n1 * n1; ++i) T.k1s[i] = std::pow(L.h, d - 2) * K1[i];
    }
    // Patches and their inverses (levels >= 1), coarse inverse (level 0).
    for (int l = 0; l < cfg.n_levels; ++l) {
      HostLevel& L = H.levels[l];
      LevelTables& T = H.tables[l];
      LevelGeom geo{d, k, L.N, L.nn};
      std::vector<double> Gd[kMaxDim];
      for (int dir = 0; dir < d; ++dir) ghost_face_matrix(cfg, H.basis, L.h, dir, Gd[dir]);
      Assembler As{cfg, L, T.kcell, Gd, d, k, n1, nl, geo};
      if (l == 0) {
        const int n0 = static_cast<int>(L.n_dofs);
        H.n_coarse = n0;
        if (!numeric) continue;
        H.coarse_inv.assign(static_cast<size_t>(n0) * n0, 0.0);
        auto pos = [&](int64_t node) { return L.node_dof[node]; };
        for (int64_t c = 0; c < L.n_cells; ++c) {
          if (!(L.cell_flags[c] & kActive)) continue;
          int ci[kMaxDim];
          geo.cell_of(c, ci);
          As.add_cell(ci, pos, H.coarse_inv.data(), n0);
          for (int dir = 0; dir < d; ++dir)
            if (L.ghost_mask[c] & (1 << (2 * dir + 1))) As.add_face(ci, dir, pos, H.coarse_inv.data(), n0);
        }
        if (!spd_inverse(n0, H.coarse_inv.data())) return "ENOTSPD: coarse matrix A_0";
        continue;
      }
      const int NV = L.N + 1;
      const int nverts = ipow(NV, d);
      struct PatchRec { int32_t v; int colour; std::vector<int32_t> nodes; };
      std::vector<PatchRec> cutp;
      for (int c = 0; c < 8; ++c) { L.int_vertex[c].clear(); L.cut[c] = CutPatchGroup(); }
      L.n_int_patches = L.n_cut_patches = 0;
      for (int v = 0; v < nverts; ++v) {
        int V[kMaxDim];
        for (int j = 0, r = v; j < d; ++j) { V[j] = r % NV; r /= NV; }
        bool any = false, all_int = true;
        int ncell = 0;
        for (int o = 0; o < (1 << d); ++o) {
          int ci[kMaxDim];
          bool in = true;
          for (int j = 0; j < d; ++j) {
            ci[j] = V[j] - 1 + ((o >> j) & 1);
            in &= ci[j] >= 0 && ci[j] < L.N;
          }
          if (!in) { all_int = false; continue; }
          ++ncell;
          const uint8_t f = L.cell_flags[geo.cell(ci)];
          if (f & kActive) any = true;
          if (!(f & kActive) || (f & kCut)) all_int = false;
          // a cut cell across the patch boundary makes a ghost face on it
          for (int j = 0; j < d && all_int; ++j) {
            int nb[kMaxDim];
            std::memcpy(nb, ci, sizeof nb);
            nb[j] += ((o >> j) & 1) ? 1 : -1;
            if (nb[j] >= 0 && nb[j] < L.N && (L.cell_flags[geo.cell(nb)] & kCut)) all_int = false;
          }
        }
        if (!any) continue;
        all_int = all_int && ncell == (1 << d);
        int colour = 0;
        for (int j = 0; j < d; ++j) colour |= (V[j] & 1) << j;
        if (all_int) {
          L.int_vertex[colour].push_back(v);
          ++L.n_int_patches;
          continue;
        }
        PatchRec rec{v, colour, {}};
        int lo[kMaxDim], hi[kMaxDim];
        for (int j = 0; j < d; ++j) {
          lo[j] = std::max(k * V[j] - k + 1, 0);
          hi[j] = std::min(k * V[j] + k - 1, L.nn - 1);
        }
        int I[kMaxDim] = {0, 0, 0};
        if (d == 2) {
          for (I[1] = lo[1]; I[1] <= hi[1]; ++I[1])
            for (I[0] = lo[0]; I[0] <= hi[0]; ++I[0])
              if (L.node_dof[geo.node(I)] >= 0) rec.nodes.push_back(static_cast<int32_t>(geo.node(I)));
        } else {
          for (I[2] = lo[2]; I[2] <= hi[2]; ++I[2])
            for (I[1] = lo[1]; I[1] <= hi[1]; ++I[1])
              for (I[0] = lo[0]; I[0] <= hi[0]; ++I[0])
                if (L.node_dof[geo.node(I)] >= 0) rec.nodes.push_back(static_cast<int32_t>(geo.node(I)));
        }
        cutp.push_back(std::move(rec));
      }
      L.n_cut_patches = cutp.size();
      // group by colour, keep vertex order inside a colour
      std::vector<int> order[8];
      for (size_t i = 0; i < cutp.size(); ++i) order[cutp[i].colour].push_back(static_cast<int>(i));
      for (int col = 0; col < 8; ++col) {
        CutPatchGroup& g = L.cut[col];
        g.off.push_back(0);
        g.inv_off.push_back(0);
        for (int i : order[col]) {
          const auto& rec = cutp[i];
          g.vertex.push_back(rec.v);
          g.nodes.insert(g.nodes.end(), rec.nodes.begin(), rec.nodes.end());
          g.off.push_back(static_cast<int32_t>(g.nodes.size()));
          const int64_t nj = rec.nodes.size();
          g.inv_off.push_back(g.inv_off.back() + nj * nj);
        }
        std::string perr;
        const int np = numeric ? static_cast<int>(g.vertex.size()) : 0;
        g.inv.assign(numeric ? g.inv_off.back() : 0, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
        for (int p = 0; p < np; ++p) {
          const int nj = g.off[p + 1] - g.off[p];
          const int32_t* nodes = &g.nodes[g.off[p]];
          auto pos = [&](int64_t node) {
            for (int t = 0; t < nj; ++t)
              if (nodes[t] == node) return t;
            return -1;
          };
          double* A = &g.inv[g.inv_off[p]];
          int V[kMaxDim];
          for (int j = 0, r = g.vertex[p]; j < d; ++j) { V[j] = r % NV; r /= NV; }
          for (int o = 0; o < (1 << d); ++o) {
            int ci[kMaxDim];
            bool in = true;
            for (int j = 0; j < d; ++j) {
              ci[j] = V[j] - 1 + ((o >> j) & 1);
              in &= ci[j] >= 0 && ci[j] < L.N;
            }
            if (!in) continue;
            const int64_t c = geo.cell(ci);
            if (!(L.cell_flags[c] & kActive)) continue;
            As.add_cell(ci, pos, A, nj);
            for (int dir = 0; dir < d; ++dir) {
              // faces of this cell that are ghost faces; internal faces of the
              // patch are counted once, from their lower cell
              if (L.ghost_mask[c] & (1 << (2 * dir + 1))) As.add_face(ci, dir, pos, A, nj);
              if (L.ghost_mask[c] & (1 << (2 * dir + 0))) {
                const bool lower_in_patch = ((o >> dir) & 1) == 1;
                if (!lower_in_patch) {
                  int lc[kMaxDim];
                  std::memcpy(lc, ci, sizeof lc);
                  lc[dir] -= 1;
                  As.add_face(lc, dir, pos, A, nj);
                }
              }
            }
          }
          if (!spd_inverse(nj, A)) {
#pragma omp critical
            perr = "ENOTSPD: local matrix of a cut patch";
          }
        }
        if (!perr.empty()) return perr;
      }
      cut_step_sets(L, d, k);
    }
  } catch (const std::exception& ex) {
    return std::string("EINVAL: ") + ex.what();
  }
  return "";
}

// Node sets of the cut colour steps of one level: the cut region (every active
// node a cut step reads: the closure of each cut patch and the cells across its
// ghost faces, i.e. cells V-2 and V+1 along one direction) and, per colour, which
// internal DoFs are also internal DoFs of the next / previous colour that has
// cut patches.
void cut_step_sets(HostLevel& L, int d, int k) {
  LevelGeom geo{d, k, L.N, L.nn};
  const int NV = L.N + 1;
  std::vector<uint8_t> member(static_cast<size_t>(L.n_nodes), 0), region(static_cast<size_t>(L.n_nodes), 0);
  int present[8], np = 0;
  for (int c = 0; c < 8; ++c) {
    for (int32_t n : L.cut[c].nodes) member[n] |= static_cast<uint8_t>(1u << c);
    if (!L.cut[c].vertex.empty()) present[np++] = c;
  }
  const int span = 4;  // cells V-2 .. V+1 per direction
  for (int c = 0; c < 8; ++c)
    for (int32_t v : L.cut[c].vertex) {
      int V[kMaxDim];
      for (int j = 0, r = v; j < d; ++j) { V[j] = r % NV; r /= NV; }
      for (int o = 0; o < ipow(span, d); ++o) {
        int ci[kMaxDim], outer = 0;
        bool in = true;
        for (int j = 0, r = o; j < d; ++j, r /= span) {
          const int t = r % span;
          ci[j] = V[j] - 2 + t;
          outer += t == 0 || t == span - 1;
          in &= ci[j] >= 0 && ci[j] < L.N;
        }
        if (!in || outer > 1) continue;
        int I[kMaxDim] = {0, 0, 0};
        for (int q = 0; q < ipow(k + 1, d); ++q) {
          for (int j = 0, r = q; j < d; ++j, r /= k + 1) I[j] = k * ci[j] + r % (k + 1);
          region[geo.node(I)] = 1;
        }
      }
    }
  L.cut_region.clear();
  for (int64_t n = 0; n < L.n_nodes; ++n)
    if (region[n] && L.node_dof[n] >= 0) L.cut_region.push_back(static_cast<int32_t>(n));
  for (int i = 0; i < np; ++i) {
    const int c = present[i], fwd = present[(i + 1) % np], bwd = present[(i + np - 1) % np];
    CutPatchGroup& g = L.cut[c];
    g.nxt.resize(g.nodes.size());
    for (size_t t = 0; t < g.nodes.size(); ++t) {
      const uint8_t m = member[g.nodes[t]];
      g.nxt[t] = static_cast<uint8_t>(((m >> fwd) & 1) | (((m >> bwd) & 1) << 1));
    }
  }
}

void manufactured_rhs(const Hierarchy& H, std::vector<double>& b) {
  const int d = H.cfg.dim;
  auto u = [d](const double* x) {
    double v = 1.0;
    for (int j = 0; j < d; ++j) v *= std::sin(M_PI * x[j]);
    return v;
  };
  load_vector(H, [&](const double* x) { return d * M_PI * M_PI * u(x); }, u, b);
}

void fourier_rhs(const Hierarchy& H, int n_modes, const int* kappa, const double* amp, const double* phase,
                 std::vector<double>& b) {
  const int d = H.cfg.dim;
  int kmax = 0;
  for (int i = 0; i < n_modes * d; ++i) kmax = std::max(kmax, std::abs(kappa[i]));
  constexpr int kTab = 16;
  if (kmax > kTab) {  // direct evaluation
    auto f = [&](const double* x) {
      double v = 0.0;
      for (int q = 0; q < n_modes; ++q) {
        double arg = phase[q];
        for (int j = 0; j < d; ++j) arg += M_PI * kappa[q * d + j] * x[j];
        v += amp[q] * std::cos(arg);
      }
      return v;
    };
    load_vector(H, f, nullptr, b);
    return;
  }
  // cos(pi kappa.x + theta) = Re(e^{i theta} prod_j e^{i pi kappa_j x_j}): two
  // trigonometric calls per direction and point, the multiples of pi x_j by
  // the angle-addition recurrence, a few products per mode
  std::vector<double> cth(n_modes), sth(n_modes);
  for (int q = 0; q < n_modes; ++q) {
    cth[q] = std::cos(phase[q]);
    sth[q] = std::sin(phase[q]);
  }
  auto f = [&](const double* x) {
    double c[kMaxDim][kTab + 1], sn[kMaxDim][kTab + 1];
    for (int j = 0; j < d; ++j) {
      const double c1 = std::cos(M_PI * x[j]), s1 = std::sin(M_PI * x[j]);
      c[j][0] = 1.0;
      sn[j][0] = 0.0;
      for (int m = 0; m < kmax; ++m) {
        c[j][m + 1] = c[j][m] * c1 - sn[j][m] * s1;
        sn[j][m + 1] = sn[j][m] * c1 + c[j][m] * s1;
      }
    }
    double v = 0.0;
    for (int q = 0; q < n_modes; ++q) {
      double re = cth[q], im = sth[q];
      for (int j = 0; j < d; ++j) {
        const int kq = kappa[q * d + j], ka = std::abs(kq);
        const double cr = c[j][ka], ci = kq < 0 ? -sn[j][ka] : sn[j][ka];
        const double t = re * cr - im * ci;
        im = re * ci + im * cr;
        re = t;
      }
      v += amp[q] * re;
    }
    return v;
  };
  load_vector(H, f, nullptr, b);
}

void build_rhs_plan(const Hierarchy& H, RhsPlan& R) {
  const Config& cfg = H.cfg;
  const HostLevel& L = H.levels.back();
  const int d = cfg.dim;
  LevelGeom geo{d, cfg.k, L.N, L.nn};
  R = RhsPlan{};
  R.act_id.assign(static_cast<size_t>(L.n_cells), -1);
  for (int64_t c = 0; c < L.n_cells; ++c) {
    if (!(L.cell_flags[c] & kActive)) continue;
    R.act_id[c] = static_cast<int32_t>(R.n_active++);
    if (L.cell_flags[c] & kCut) R.cut.push_back(static_cast<int32_t>(c));
    else R.uncut.push_back(static_cast<int32_t>(c));
  }
  // columns per cut cell in parallel, concatenated in cut-cell order
  const int64_t nc = static_cast<int64_t>(R.cut.size());
  std::vector<std::vector<Column>> per(static_cast<size_t>(nc));
  const int nq = cfg.quad_n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nc; ++i) {
    int ci[kMaxDim];
    geo.cell_of(R.cut[i], ci);
    double lo[kMaxDim], hi[kMaxDim];
    for (int j = 0; j < d; ++j) { lo[j] = cfg.lo + ci[j] * L.h; hi[j] = lo[j] + L.h; }
    std::vector<Column> cols;
    cut_columns_union(d, cfg.shapes, lo, hi, nq, nq, cfg.quad_beta, cfg.union_depth, cols);
    for (const Column& col : cols)
      if (col.t1 > col.t0) per[i].push_back(col);
  }
  R.col_off.assign(static_cast<size_t>(nc) + 1, 0);
  for (int64_t i = 0; i < nc; ++i) R.col_off[i + 1] = R.col_off[i] + static_cast<int64_t>(per[i].size());
  const int64_t n = R.col_off[nc];
  R.cx.resize(static_cast<size_t>(d * n));
  R.cw.resize(n);
  R.ct0.resize(n);
  R.ct1.resize(n);
  R.ce.resize(n);
  for (int64_t i = 0; i < nc; ++i)
    for (size_t t = 0; t < per[i].size(); ++t) {
      const Column& col = per[i][t];
      const int64_t o = R.col_off[i] + static_cast<int64_t>(t);
      for (int j = 0; j < d; ++j) R.cx[j * n + o] = col.x[j];
      R.cw[o] = col.w;
      R.ct0[o] = col.t0;
      R.ct1[o] = col.t1;
      R.ce[o] = static_cast<uint8_t>(col.e);
    }
}

void load_vector(const Hierarchy& H, const std::function<double(const double*)>& f,
                 const std::function<double(const double*)>& u, std::vector<double>& b) {
  const Config& cfg = H.cfg;
  const HostLevel& L = H.levels.back();
  const int d = cfg.dim, k = cfg.k, n1 = k + 1, nl = ipow(n1, d);
  LevelGeom geo{d, k, L.N, L.nn};
  const double h = L.h;
  b.assign(L.n_dofs, 0.0);
  const int ng = k + 3;
  double gx[16], gw[16];
  gauss_legendre(ng, gx, gw);
  const int nq = cfg.quad_n;
  std::vector<double> tx(nq), tw(nq);
  gauss_legendre(nq, tx.data(), tw.data());
  std::vector<int64_t> cells;
  for (int64_t c = 0; c < L.n_cells; ++c)
    if (L.cell_flags[c] & kActive) cells.push_back(c);
  // cell vectors in parallel, then summed into b in cell order (deterministic)
  std::vector<double> locs(cells.size() * static_cast<size_t>(nl), 0.0);
#pragma omp parallel
  {
    // 1-D basis values (and derivatives) at the point, per direction
    double e[kMaxDim][kMaxDeg + 1], de[kMaxDim][kMaxDeg + 1];
    auto tabulate = [&](const double* xi, bool deriv) {
      for (int j = 0; j < d; ++j)
        for (int i = 0; i < n1; ++i) {
          e[j][i] = H.basis.eval(i, xi[j], 0);
          if (deriv) de[j][i] = H.basis.eval(i, xi[j], 1);
        }
    };
    auto phi = [&](int a, int deriv_dir) {
      double v = 1.0;
      for (int j = 0, r = a; j < d; ++j) {
        v *= j == deriv_dir ? de[j][r % n1] : e[j][r % n1];
        r /= n1;
      }
      return v;
    };
    std::vector<Column> cols;
#pragma omp for schedule(dynamic, 16)
    for (int64_t ic = 0; ic < static_cast<int64_t>(cells.size()); ++ic) {
      const int64_t c = cells[ic];
      double* loc = locs.data() + ic * nl;
      int ci[kMaxDim];
      geo.cell_of(c, ci);
      double lo[kMaxDim], hi[kMaxDim];
      for (int j = 0; j < d; ++j) { lo[j] = cfg.lo + ci[j] * h; hi[j] = lo[j] + h; }
      if (!(L.cell_flags[c] & kCut)) {
        const int npts = ipow(ng, d);
        for (int p = 0; p < npts; ++p) {
          double xi[kMaxDim], x[kMaxDim], w = std::pow(h, d);
          for (int j = 0, r = p; j < d; ++j) { xi[j] = gx[r % ng]; w *= gw[r % ng]; x[j] = lo[j] + h * xi[j]; r /= ng; }
          const double fv = f(x) * w;
          tabulate(xi, false);
          for (int a = 0; a < nl; ++a) loc[a] += fv * phi(a, -1);
        }
        continue;
      }
      cols.clear();
      cut_columns_union(d, cfg.shapes, lo, hi, nq, nq, cfg.quad_beta, cfg.union_depth, cols);
      for (const Column& col : cols) {
        double x[kMaxDim], xi[kMaxDim];
        for (int j = 0; j < d; ++j) x[j] = col.x[j];
        if (col.t1 > col.t0) {
          // along the column only direction e varies: the basis factors of the
          // other directions are tabulated once, and each point adds
          // f w psi_{a_e}(xi_e) into a per-(tangential index, a_e) sum
          for (int j = 0; j < d; ++j) xi[j] = (x[j] - lo[j]) / h;
          tabulate(xi, false);
          double acc[kMaxDeg + 1] = {};
          double ee[kMaxDeg + 1];
          for (int t = 0; t < nq; ++t) {
            x[col.e] = col.t0 + (col.t1 - col.t0) * tx[t];
            const double fv = f(x) * col.w * (col.t1 - col.t0) * tw[t];
            const double xe = (x[col.e] - lo[col.e]) / h;
            for (int i = 0; i < n1; ++i) ee[i] = H.basis.eval(i, xe, 0);
            for (int i = 0; i < n1; ++i) acc[i] += fv * ee[i];
          }
          for (int a = 0; a < nl; ++a) {
            double v = 1.0;
            int ae = 0;
            for (int j = 0, r = a; j < d; ++j) {
              if (j == col.e) ae = r % n1;
              else v *= e[j][r % n1];
              r /= n1;
            }
            loc[a] += v * acc[ae];
          }
        }
        if (col.surf && u) {
          x[col.e] = col.ts;
          for (int j = 0; j < d; ++j) xi[j] = (x[j] - lo[j]) / h;
          const double gv = u(x) * col.sw;
          tabulate(xi, true);
          for (int a = 0; a < nl; ++a) {
            double dn = 0.0;
            for (int j = 0; j < d; ++j) dn += col.nrm[j] * phi(a, j) / h;
            loc[a] += gv * (cfg.gamma_D / h * phi(a, -1) - dn);
          }
        }
      }
    }
  }
  for (size_t ic = 0; ic < cells.size(); ++ic) {
    int ci[kMaxDim];
    geo.cell_of(cells[ic], ci);
    for (int a = 0; a < nl; ++a) {
      int I[kMaxDim];
      for (int j = 0, r = a; j < d; ++j) { I[j] = k * ci[j] + r % n1; r /= n1; }
      b[L.node_dof[geo.node(I)]] += locs[ic * nl + a];
    }
  }
}

}  // namespace cmg
