// Device-side views of one multigrid level and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include <cstdint>

namespace cmg {

// One level as seen by the kernels (all pointers are device pointers).
struct KLevel {
  int N;                     // cells per direction
  int nn;                    // lattice nodes per direction, k N + 1
  int64_t n_dofs;
  int64_t n_nodes;           // lattice nodes, nn^d (the column stride of lattice vectors)
  const uint8_t* flags;      // per cell: bit 0 active, bit 1 cut
  const int32_t* cut_id;     // per cell: index of its cut-cell matrix or -1
  const uint8_t* ghost;      // per cell: bit 2*dir+side marks a ghost face
  const void* cut_mats;      // n_cut x (k+1)^d x (k+1)^d, scalar type of the path (symmetric)
  const void* cut_packed;    // the same matrices as upper triangles, row-major, (k+1)^d ((k+1)^d + 1) / 2 each
  int64_t n_cut;             // cut cells
  const int32_t* dof_node;   // lattice node of each DoF, ascending
  const double* tables;      // constant tables (uncut stiffness, 1-D factors, FD, prolongation)
  const float* kcell32;      // FP32 path: the uncut cell stiffness of the tables rounded to FP32 (else null)
  int64_t n_faces;           // ghost faces
  const int32_t* face_lower; // lower cell of every ghost face
  const uint8_t* face_dir;   // its normal direction
  const int32_t* cell_gid;   // per cell: row of cell_faces or -1
  const int32_t* cell_faces; // 2d face ids per cell with ghost faces (-1: none)
  int n_tiles;               // operator tiles owning active nodes whose staged cells (-1 .. B-1 around
  const int32_t* tiles;      // the tile) include a special or inactive cell: dense rows and pre-pass values
  int n_tiles_sf;            // the other tiles owning active nodes: every staged cell active and regular,
  const int32_t* tiles_sf;   // applied by sum factorisation
  int64_t n_spec;            // special cells: cut, or with a ghost face
  const int32_t* spec_cells; // background cell of every special cell
  const int32_t* spec_info;  // per special cell 1 + 2d entries: cut id (-1: uncut), ghost face ids (-1: none)
  const int32_t* cell_sid;   // per cell: special id, -1 active and regular, -2 inactive
  int ghost_local;           // cut colour steps: 1 = x beyond the patch closure is taken as zero (the ghost
                             // faces on the patch boundary contribute only their closure part), 0 = exact
  template <typename T>
  __host__ __device__ const T* cut_mats_t() const { return static_cast<const T*>(cut_mats); }
  // the uncut cell stiffness (row-major (k+1)^d x (k+1)^d) in the path's precision
  template <typename T>
  __host__ __device__ const T* kcell_t() const {
    if constexpr (sizeof(T) == 4) return kcell32;
    else return tables;
  }
  template <typename T>
  __host__ __device__ const T* cut_packed_t() const { return static_cast<const T*>(cut_packed); }
};

// Cut patches of one colour.
struct CutGroupDev {
  int n_patch;
  int64_t n_nodes;
  const int32_t* off;        // node offsets, n_patch + 1
  const int64_t* inv_off;    // inverse offsets, n_patch + 1
  const int32_t* nodes;      // lattice nodes of the internal DoFs
  const int32_t* vertex;     // vertex index of every patch
  const int32_t* cell_cut;   // per patch and cell o of its 2^d: cut-cell index, -1 if uncut or outside
  const uint16_t* cell_fg;   // per patch and cell o: flags | ghost bits << 8 (0 outside the box)
  const void* inv;           // symmetric dense inverses, scalar type of the path
  const float* inv_tiles;    // FP32 inverses in MFMA tile order (see k_cut_solve_mfma), or null
  const int64_t* tile_off;   // tile offsets, n_patch + 1, or null
  const uint8_t* nxt;        // per node: bit 0 (1) also internal to the next (previous) cut colour
  template <typename T>
  __host__ __device__ const T* inv_t() const { return static_cast<const T*>(inv); }
};

// Copy part of a two-buffer cut step: dst[nodes[i]] = src[nodes[i]] for the i < n
// whose skip[i] has none of the bits of mask, in nblk extra blocks placed before
// the patch blocks (the launcher sets nblk for its block size).
struct CopyJob {
  const int32_t* nodes = nullptr;
  const uint8_t* skip = nullptr;
  int mask = 0;
  int64_t n = 0;
  int nblk = 0;
};

constexpr int kMaxCols = 8;  // columns (right-hand sides) of one multi-column launch

// Launch shape choices that depend on the size of a launch, settable per
// problem so that tests can force the configuration a large level runs in on
// a small one.  Results do not depend on them beyond rounding-free choices:
// the arithmetic of every node is the same for any block size and grid cap.
struct LaunchPolicy {
  int small_cut_launch = 1536;  // cut colour steps with fewer patches use twice the threads per patch block
  unsigned max_blocks = 2048;   // grid cap of the grid-stride kernels (operator tiles, interior patches)
};

// Per-column coefficients of the column-wise vector kernels.
struct ColCoef {
  double v[kMaxCols];
};

constexpr int kMaxRows = 64;  // rows of one row combination (Krylov basis vectors)

struct RowCoef {
  double v[kMaxRows];
};

int tables_size(int d, int k);

// Grouped launches.  While a recorder is set on the calling thread, the
// multigrid launchers below append their launches to it instead of issuing
// them: the grouped form of the kernel (one launch over several problems,
// blockIdx.z selecting the problem's argument record in a device table), the
// block grid and block size of this problem's launch and its argument record.
// Launches without a grouped form append an empty record (fn == nullptr).
// While recording, the operator pre-passes, interior colour steps and zero
// fills are recorded also where they have no work, so that problems of one
// lattice shape record the same sequence of kernels.
struct LaunchRecord {
  const void* fn = nullptr;
  unsigned grid[2] = {0, 0};
  unsigned block = 0;
  std::vector<unsigned char> args;
};
void set_launch_recorder(std::vector<LaunchRecord>* rec);  // nullptr: launch again
bool launch_recording();

// Every multigrid launcher works on ncol columns at once (blockIdx.y = column):
// lattice vectors of a level are ncol blocks of KLevel::n_nodes entries, the
// ghost-face work buffer ncol blocks of n_faces k (k+1)^(d-1) entries, the
// cut-patch correction buffer ncol blocks of CutGroupDev::n_nodes entries, and
// compact (DoF-ordered) vectors ncol blocks of n entries.

// y = A x (b == nullptr) or y = b - A x on every active node; W is the work
// buffer for the ghost-face jumps, C the one for the special-cell products
// (n_spec (k+1)^d entries per column).
template <typename T>
hipError_t launch_apply(int d, int k, const KLevel& L, const T* x, const T* b, T* y, T* W, T* C, hipStream_t s,
                        int ncol = 1, const LaunchPolicy& lp = LaunchPolicy());
template <typename T>
hipError_t launch_interior_step(int d, int k, const KLevel& L, const int32_t* verts, int nv, T* x, const T* b,
                                hipStream_t s, int ncol = 1, const LaunchPolicy& lp = LaunchPolicy());
// Cut colour step, phase 1.  xb == nullptr: the corrections d_j go to dbuf
// (launch_cut_update adds them).  Otherwise two-buffer form: x is read, and
// xb receives x + d_j on the internal DoFs of the colour plus the copy job
// (build it with cut_copy_job; x and xb are distinct buffers).
template <typename T>
hipError_t launch_cut_solve(int d, int k, const KLevel& L, const CutGroupDev& G, const T* x, const T* b, T* dbuf,
                            hipStream_t s, int ncol = 1, T* xb = nullptr, const CopyJob& cj = CopyJob(),
                            const LaunchPolicy& lp = LaunchPolicy());
// Copy job of a two-buffer step after the step of colour group Gp: the nodes of
// Gp that are not internal to the current colour (mask 1: next colour in
// increasing order, 2: in decreasing order).
CopyJob cut_copy_job(int d, int k, const CutGroupDev& Gp, int mask);
// dst[nodes[i]] = src[nodes[i]] (ncol columns, ld apart)
template <typename T>
hipError_t launch_copy_nodes(const int32_t* nodes, int64_t n, const T* src, T* dst, int64_t ld, hipStream_t s,
                             int ncol = 1);
// FP32, ncol <= kMaxCols columns, local solves on the matrix cores (needs
// inv_tiles); W is the ghost-face work buffer (ncol columns), rewritten here.
// FP64 counterpart for several columns: every inverse and cell row read once
// for all columns (plain FMA); corrections into dbuf like the FP32 kernel.
hipError_t launch_cut_solve_cols(int d, int k, const KLevel& L, const CutGroupDev& G, const double* x,
                                 const double* b, double* W, double* dbuf, int ncol, hipStream_t s);
hipError_t launch_cut_solve_mfma(int d, int k, const KLevel& L, const CutGroupDev& G, const float* x, const float* b,
                                 float* W, float* dbuf, int ncol, hipStream_t s);
template <typename T>
hipError_t launch_cut_update(const CutGroupDev& G, const T* dbuf, T* x, int64_t ldx, hipStream_t s, int ncol = 1);
template <typename T>
hipError_t launch_prolong_add(int d, int k, const KLevel& Lc, const KLevel& Lf, const T* xc, T* xf, hipStream_t s,
                              int ncol = 1);
template <typename T>
hipError_t launch_restrict(int d, int k, const KLevel& Lc, const KLevel& Lf, const T* rf, T* bc, hipStream_t s,
                           int ncol = 1);
template <typename T>
hipError_t launch_coarse(const T* inv, const int32_t* dof_node, int n0, const T* b, T* x, int64_t ld, hipStream_t s,
                         int ncol = 1);
template <typename T>
hipError_t launch_zero_active(const int32_t* dof_node, int64_t n, T* x, int64_t ld, hipStream_t s, int ncol = 1);
template <typename TS, typename TD>
hipError_t launch_scatter(const int32_t* dof_node, int64_t n, const TS* src, TD* lat, int64_t ld, hipStream_t s,
                          int ncol = 1);
template <typename TS, typename TD>
hipError_t launch_gather(const int32_t* dof_node, int64_t n, const TS* lat, TD* dst, int64_t ld, hipStream_t s,
                         int ncol = 1);

}  // namespace cmg

namespace cmg {
// part[c * nblk + i]: partial sums of column c (ncol columns of n entries)
hipError_t launch_dot_partial(const double* x, const double* y, int64_t n, double* part, int nblk, hipStream_t s,
                              int ncol = 1);
hipError_t launch_axpy_cols(int64_t n, const ColCoef& a, const double* x, double* y, int ncol, hipStream_t s);
// part[j * nblk + i]: partial sums of V_j . w for the m rows of V (n entries each)
hipError_t launch_rows_dot_partial(const double* V, const double* w, int64_t n, int m, double* part, int nblk,
                                   hipStream_t s);
// y += sum_{j < m} c.v[j] V_j
hipError_t launch_rows_combine(int64_t n, int m, const RowCoef& c, const double* V, double* y, hipStream_t s);
hipError_t launch_scale(int64_t n, double a, const double* x, double* y, hipStream_t s);  // y = a x
hipError_t launch_xpay_cols(int64_t n, const ColCoef& a, const double* x, double* y, int ncol, hipStream_t s);
hipError_t launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s);   // y += a x
hipError_t launch_xpay(int64_t n, double a, const double* x, double* y, hipStream_t s);   // y = x + a y
}  // namespace cmg

namespace cmg {
// Held by every device allocation, null-stream upload or device-wide
// synchronisation of the library and by the capture of V-cycle graphs, so
// that the two never overlap across threads (api.cpp).
std::recursive_mutex& device_mutex();

// Load vector of f = sum_q amp_q cos(pi kappa_q . x + phase_q) with g = 0 on
// the finest level, assembled on the device from the quadrature plan of the
// host set-up (cell vectors of every active cell, then one gather per DoF;
// every sum in a fixed order, so the result is the same in every run).
constexpr int kMaxModes = 32;
struct RhsModes {
  int n;
  int kappa[kMaxModes][3];
  double amp[kMaxModes], phase[kMaxModes];
};
struct RhsPlanDev {
  int N, nn;                 // cells / lattice nodes per direction
  double lo, h;              // box corner and cell size
  int64_t n_uncut, n_cut, n_col;
  const int32_t* uncut;      // background cells of the active uncut cells
  const int32_t* cut;        // background cells of the cut cells
  const int64_t* col_off;    // volume columns of cut cell i: col_off[i] .. col_off[i+1]
  const double* cx;          // base points, SoA (dim arrays of n_col)
  const double* cw;
  const double* ct0;
  const double* ct1;
  const uint8_t* ce;         // height direction of every column
  const int32_t* act_id;     // per background cell: row of loc, -1 inactive
  double* loc;               // cell vectors, (k+1)^d per active cell
  double coef[4][4];         // monomial coefficients of the 1-D GLL basis, psi_a(t) = sum_m coef[a][m] t^m
  double gx[8], gw[8];       // k+3 Gauss points / weights on [0, 1] (uncut cells)
  double tx[16], tw[16];     // quad_n points / weights on [0, 1] (along a column)
  int nq;
};
hipError_t launch_rhs_fourier(int d, int k, const RhsPlanDev& R, const RhsModes& M, const int32_t* dof_node,
                              int64_t n_dofs, double* b, hipStream_t s);

// Scratch of cmg_apply_noalloc: one file-scope device array per device, held
// for the life of the process.  noalloc_scratch_init, called with the device
// current (at set-up), takes its device address with hipGetSymbolAddress once
// per device; noalloc_scratch returns that address (nullptr before the init).
constexpr size_t kNoallocScratchBytes = size_t(32) << 20;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);
hipError_t launch_fill(int64_t n, double v, double* y, hipStream_t s);                    // y = v
hipError_t launch_copy(int64_t n, const double* x, double* y, hipStream_t s);             // y = x
}  // namespace cmg
