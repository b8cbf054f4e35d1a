// Host-side (CPU) set-up of the CutFEM vertex-patch multigrid hierarchy.
//
// The paper computes geometry, cut-cell quadrature and the local matrices of cut
// patches upfront on the CPU and loads them to the GPU (Section 3).  This header
// declares that set-up: 1-D Q_k basis on Gauss-Lobatto points, dimension-
// reduction quadrature on cut cells, element matrices of the Nitsche form with
// face ghost penalties, vertex patches with colours, FP64 local inverses and the
// per-level constant tables the HIP kernels use.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace cmg {

constexpr int kMaxDim = 3;
constexpr int kMaxDeg = 3;

enum CellFlag : uint8_t { kActive = 1, kCut = 2 };

struct Shape {            // axis-aligned ellipsoid  sum_j ((x_j - c_j)/s_j)^2 < 1
  double c[kMaxDim] = {0, 0, 0};
  double s[kMaxDim] = {1, 1, 1};
};

struct Config {
  int dim = 2, k = 2, n_levels = 2, coarse_cells = 4;
  double lo = -1.0, hi = 1.0;
  std::vector<Shape> shapes;
  double gamma_D = 120.0, gamma_g = 0.1;
  double gamma_m[3] = {0.0, 0.0, 0.0};  // per derivative order; <= 0: gamma_g
  double gamma(int m) const { return gamma_m[m - 1] > 0.0 ? gamma_m[m - 1] : gamma_g; }
  int ghost_exp_mode = 0;     // 0: h^(2m-1), 1: h^(2m+1)
  int n_c = 2;
  int quad_n = 14;            // Gauss points per smooth piece of a cut-cell rule
  double quad_beta = 0.35;    // subdivision threshold of the cut-cell rule
  int union_depth = 4;        // bisection depth of boxes crossed by several surfaces
};

// ---- 1-D basis (reference interval [0,1]) ---------------------------------
struct Basis1D {
  int k = 0;
  double node[kMaxDeg + 1];                            // GLL nodes
  double coef[kMaxDeg + 1][kMaxDeg + 1];               // monomial coefficients of psi_a
  double eval(int a, double t, int deriv = 0) const;   // psi_a^(deriv)(t)
};
Basis1D make_basis(int k);
void gauss_legendre(int n, double* x, double* w);      // on [0,1]

// ---- dense linear algebra (row-major, small) --------------------------------
// In-place inverse of an SPD matrix via Cholesky; returns false if not SPD.
bool spd_inverse(int n, double* a);
// Generalized symmetric eigenproblem K s = lambda M s, S^T M S = I (M SPD).
bool gen_eig(int n, const double* K, const double* M, double* S, double* lam);

// ---- cut-cell quadrature ------------------------------------------------------
// One vertical column of a cut-cell rule: base point, base weight, height
// direction e, the part [t0, t1] of the column inside Omega (t1 <= t0: none) and,
// if the column crosses Gamma, the crossing point with its surface weight and
// outward unit normal.
struct Column {
  int e;
  double x[kMaxDim];       // base point (component e unused)
  double w;
  double t0, t1;
  bool surf;
  double ts, sw, nrm[kMaxDim];
};
// Enumerate the columns of the rule for box [a, b] and one shape.  n: Gauss
// points per smooth piece of the base; full sub-boxes use n_full points per
// base direction.
void cut_columns(int dim, const Shape& sh, const double* a, const double* b, int n, int n_full,
                 double beta, std::vector<Column>& out);
// Same for the union of several shapes: boxes crossed by one surface use the
// single-shape rule, boxes crossed by several are bisected up to union_depth
// and then integrated column by column with exact unions of the per-shape
// intervals (a volume column per merged interval, a surface-only column per
// boundary point).
void cut_columns_union(int dim, const std::vector<Shape>& shapes, const double* a, const double* b, int n,
                       int n_full, double beta, int union_depth, std::vector<Column>& out);

// ---- hierarchy --------------------------------------------------------------
struct CutPatchGroup {          // cut patches of one colour on one level
  std::vector<int32_t> vertex;  // vertex linear index (diagnostics)
  std::vector<int32_t> off;     // offset of the patch's nodes (size n_patch + 1)
  std::vector<int64_t> inv_off; // offset of its dense inverse (size n_patch + 1)
  std::vector<int32_t> nodes;   // lattice node indices of the internal DoFs
  std::vector<double> inv;      // dense symmetric N_j x N_j inverses
  std::vector<uint8_t> nxt;     // per node: bit 0 (1) it is also an internal DoF of a cut patch of
                                // the next (previous) colour with cut patches, cyclically
};

struct HostLevel {
  int N = 0, nn = 0;            // cells / nodes per direction
  double h = 0;
  int64_t n_cells = 0, n_nodes = 0, n_dofs = 0;
  std::vector<uint8_t> cell_flags;   // per cell (x fastest)
  std::vector<int32_t> cut_id;       // per cell, -1 if not cut
  std::vector<uint8_t> ghost_mask;   // per cell: bit 2*dir+side, side 1 = upper face
  std::vector<int32_t> cell_gid;     // per cell: row of cell_faces, -1 without ghost faces
  std::vector<int32_t> cell_faces;   // 2d face ids per cell with ghost faces (-1: none)
  std::vector<int32_t> face_lower;   // ghost faces: lower cell
  std::vector<uint8_t> face_dir;     //              normal direction
  std::vector<int32_t> tiles;        // operator tiles owning active nodes (tile index, x fastest)
  std::vector<int32_t> dof_node;     // lattice node of each DoF, ascending (= canonical order)
  std::vector<int32_t> node_dof;     // per lattice node, -1 if inactive
  std::vector<double> cut_mats;      // n_cut x (k+1)^d x (k+1)^d, row-major
  int n_cut = 0;
  std::vector<int32_t> int_vertex[8];  // interior patches per colour (vertex linear index)
  CutPatchGroup cut[8];
  std::vector<int32_t> cut_region;  // active nodes that a cut colour step reads (closures and ghost halos)
  int64_t n_int_patches = 0, n_cut_patches = 0;
  double max_local_cond = 0;
};

// Per-level constant tables read by the kernels (see kernels.hip).
struct LevelTables {
  std::vector<double> kcell;     // (k+1)^d x (k+1)^d uncut cell stiffness, scaled
  std::vector<double> mhat;      // (k+1)^2 reference 1-D mass
  std::vector<double> d0, d1;    // k x (k+1): psi^(m)(0), psi^(m)(1), m = 1..k
  std::vector<double> gcoef;     // k: ghost coefficient per order incl. h scaling
  std::vector<double> fd_s;      // (2k-1)^2 fast-diagonalisation eigenvectors (row-major S)
  std::vector<double> fd_dinv;   // (2k-1)^d inverse eigenvalue sums incl. h scaling
  std::vector<double> p1d;       // (2k+1) x (k+1) prolongation weights
  std::vector<double> k1s;       // (k+1)^2 reference 1-D stiffness times h^(d-2)
};

struct Hierarchy {
  Config cfg;
  Basis1D basis;
  std::vector<HostLevel> levels;
  std::vector<LevelTables> tables;
  std::vector<double> coarse_inv;   // n_0 x n_0
  int64_t n_coarse = 0;
};

// Build everything; returns an empty string on success, else an error message
// prefixed by its status name ("EGEOM:", "ENOTSPD:", "EINVAL:").  numeric =
// false builds geometry, DoFs, ghost faces, patches and their node sets only
// (no cut-cell quadrature, no element matrices, no inverses): every count and
// size of the full set-up, for footprint estimates before the expensive part.
std::string build_hierarchy(const Config& cfg, Hierarchy& H, bool numeric = true);

// Load vector b_i = (f, phi_i)_Omega + (g, (gamma_D/h) phi_i - d_n phi_i)_Gamma on the
// finest level, canonical order; g may be empty (homogeneous Dirichlet data).
void load_vector(const Hierarchy& H, const std::function<double(const double*)>& f,
                 const std::function<double(const double*)>& g, std::vector<double>& b);
// Manufactured problem u = prod sin(pi x_j), f = d pi^2 u, Dirichlet data g = u.
void manufactured_rhs(const Hierarchy& H, std::vector<double>& b);
// f = sum_q amp_q cos(pi kappa_q . x + phase_q), g = 0 (kappa: n_modes x dim ints).
void fourier_rhs(const Hierarchy& H, int n_modes, const int* kappa, const double* amp, const double* phase,
                 std::vector<double>& b);

// Quadrature plan of the finest level's load vector for data with g = 0, for
// assembling it on the device: the active cells (uncut ones take the tensor
// Gauss rule with k+3 points per direction) and the volume columns of the cut
// cells' rule (the same columns as load_vector, quad_n points per smooth piece
// of the base and along every column).
struct RhsPlan {
  std::vector<int32_t> act_id;   // per background cell: row of the cell vectors, -1 inactive
  int64_t n_active = 0;
  std::vector<int32_t> uncut;    // background cells of the active uncut cells
  std::vector<int32_t> cut;      // background cells of the cut cells
  std::vector<int64_t> col_off;  // volume columns of cut cell i: col_off[i] .. col_off[i+1]
  std::vector<double> cx;        // base points, SoA: dim arrays of n_col (component e unused)
  std::vector<double> cw, ct0, ct1;  // base weight, inside interval along e
  std::vector<uint8_t> ce;       // height direction e
};
void build_rhs_plan(const Hierarchy& H, RhsPlan& R);

// Uncut-cell stiffness, element matrix of a cut cell, ghost-face matrix.
void uncut_cell_matrix(const Config& cfg, const Basis1D& B, double h, std::vector<double>& K);
void cut_cell_matrix(const Config& cfg, const Basis1D& B, double h, const double* lo,
                     std::vector<double>& E);
void ghost_face_matrix(const Config& cfg, const Basis1D& B, double h, int dir, std::vector<double>& G);

}  // namespace cmg
