/*
 * cutmg - C ABI of the CutFEM vertex-patch multigrid for AMD MI355X (gfx950).
 *
 * Problem (Cui & Kanschat, "A multigrid method for CutFEM and its
 * implementation on GPU", Section 2.1): Poisson's equation on a domain Omega
 * cut from a Cartesian background box, discretised by continuous Q_k elements
 * on the active cells (cells meeting Omega), Dirichlet data imposed by
 * Nitsche's method (eq. (cutfem_nitsche)) and face ghost penalties on the faces
 * next to cut cells (eq. (cutfem-ghost)).  The solver is the V-cycle of
 * Section 2.2 with the coloured multiplicative vertex-patch smoother of
 * Section 2.3 / eq. (smoother-split), used as preconditioner of CG.
 *
 * Conventions for every call below:
 *  - Vectors are device pointers (HBM) to float64 arrays in the canonical DoF
 *    order of their level: lexicographic on the (kN+1)^d Gauss-Lobatto node
 *    lattice (x fastest) restricted to the nodes of active cells.  Sizes come
 *    from cmg_ndofs.  The caller owns them; they must not alias unless stated.
 *  - stream is a hipStream_t (NULL = default stream).  Every device call is
 *    stream ordered and returns without synchronising, except cmg_solve, which
 *    synchronises to test convergence.
 *  - The library owns the hierarchy (geometry, matrices, patch inverses) in
 *    device memory from cmg_setup until cmg_destroy.  Internal work vectors
 *    are per problem: calls on one problem must not overlap in time.
 *  - Errors: a negative cmg_status; the message of the failing call is
 *    available from cmg_last_error() in the same thread.  Nothing is launched
 *    when argument checks fail.
 */
#ifndef CUTMG_H
#define CUTMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CMG_OK = 0,
  CMG_EINVAL = -1,     /* bad argument, unsupported shape set, level out of range */
  CMG_ENOMEM = -2,     /* device allocation failed */
  CMG_EGEOM = -3,      /* no active cell on level 0, or an active cell without active parent */
  CMG_ENOTSPD = -4,    /* Cholesky of a cut-patch or the coarse matrix failed */
  CMG_ENOTCONV = -5,   /* CG reached maxit; x holds the last iterate */
  CMG_EBREAKDOWN = -6, /* CG breakdown: p^T A p <= 0 or not finite */
  CMG_EHIP = -7,       /* a HIP runtime call failed */
  CMG_PENDING = 1      /* cmg_poll: the request has not finished yet */
} cmg_status;

typedef struct cmg_problem cmg_problem;

/* Omega = union of axis-aligned ellipsoids sum_j ((x_j - c_ij)/s_ij)^2 < 1 (a
 * sphere has equal semi-axes); host arrays of n_shapes * dim doubles.  The
 * background box is [box_lo, box_hi]^dim. */
typedef struct {
  int dim;               /* 2 or 3 */
  int n_shapes;          /* 1..16; Omega is their union (kinked where two surfaces meet) */
  const double* centers;
  const double* semi;
  double box_lo, box_hi;
} cmg_levelset;

/* Discretisation and smoother parameters (paper Section 2 and Section 4). */
typedef struct {
  int k;                 /* polynomial degree, 1..3 */
  int n_levels;          /* levels 0..n_levels-1, N_l = coarse_cells * 2^l cells per direction */
  int coarse_cells;      /* cells per direction on level 0 */
  double gamma_D;        /* Nitsche penalty: the boundary term is gamma_D / h */
  double gamma_g;        /* ghost penalty for every derivative order m = 1..k */
  int ghost_exp_mode;    /* 0: face weight h^(2m-1) / (m!)^2;  1: h^(2m+1) / (m!)^2 */
  int n_c;               /* sweeps over the cut patches per smoothing step (eq. (smoother-split)) */
  int quad_n;            /* Gauss points per smooth piece of a cut-cell rule (e.g. 14) */
  int precond_fp32;      /* 1: the V-cycle runs in FP32 (see cmg_set_precision) */
  double gamma_m[3];     /* ghost penalty of derivative order m = 1, 2, 3 (the paper tunes them one by one,
                            Section 4); an entry <= 0 means gamma_g */
} cmg_params;

typedef struct {
  int iterations;        /* CG iterations = number of V-cycle applications */
  double rel_residual;   /* final ||b - A x||_2 / ||b||_2 */
  double n_frac;         /* fractional iteration count n_it * log10(rtol) / log10(rel_residual) */
} cmg_solve_info;

/* Build the level hierarchy on the host and upload it to the current HIP
 * device (paper Section 2.1 for the nested levels, active and cut cells and
 * the discrete spaces; Section 3 for the upfront CPU part: cut-cell quadrature,
 * element matrices, and the local matrices of the cut vertex patches of
 * Section 2.3, here inverted in FP64 by Cholesky; Section 2.2 for the exact
 * coarse solver, here a dense inverse of A_0).  ls and prm are read only
 * during the call.  Synchronous: returns when the device copies are complete.
 * On success *out owns all host and device data until cmg_destroy.  Errors:
 * CMG_EINVAL (bad arguments), CMG_EGEOM (no active cell on level 0, or an
 * active cell whose parent is not active), CMG_ENOTSPD (a local or the coarse
 * matrix is not positive definite), CMG_ENOMEM, CMG_EHIP; nothing is kept. */
cmg_status cmg_setup(const cmg_levelset* ls, const cmg_params* prm, cmg_problem** out);

/* Device footprint of the problem that cmg_setup would build, without
 * building it: classifies the cells of every level and enumerates DoFs, ghost
 * faces and vertex patches with their node sets (the cheap part of the
 * set-up), but computes no cut-cell quadrature, element matrix or inverse.
 * *bytes receives exactly what cmg_device_bytes(flags) reports after
 * cmg_setup; n_dofs (may be NULL) the finest level's DoF count.  For callers
 * that admit work by memory before paying for the set-up (the solve server).
 * Host only, thread safe.  Errors as cmg_setup (CMG_EINVAL, CMG_EGEOM). */
cmg_status cmg_footprint(const cmg_levelset* ls, const cmg_params* prm, int flags, size_t* bytes, int64_t* n_dofs);

/* Same set-up without any device work (no HIP call): for inspecting the
 * hierarchy with cmg_export on machines without a GPU.  Device calls on such a
 * problem return CMG_EINVAL. */
cmg_status cmg_setup_host(const cmg_levelset* ls, const cmg_params* prm, cmg_problem** out);

/* Make a problem from cmg_setup_host device-resident on the current HIP device
 * (no-op for a device problem).  Synchronous. */
cmg_status cmg_upload(cmg_problem* p);

/* Device memory in bytes that the problem occupies once uploaded.  flags bit 0:
 * include the FP32 copies of the mixed-precision V-cycle; bit 1: include the
 * buffers of the multi-column calls (8 columns of work vectors on every level,
 * the multi-column Krylov vectors and, with bit 0, the tiled FP32 inverses);
 * bit 2: include the quadrature plan of cmg_rhs_fourier_device once it has been
 * built (zero before its first call). */
cmg_status cmg_device_bytes(const cmg_problem* p, int flags, size_t* bytes);

/* Precision of the multigrid part: fp32 = 0 runs every V-cycle kernel in FP64;
 * fp32 = 1 runs smoother, transfers, level residuals and the coarse solve in FP32
 * on FP32 copies of the cut-cell matrices and of the local and coarse inverses,
 * which are computed in FP64 and rounded (uploaded on first use).  CG
 * (cmg_solve), its operator products and all ABI vectors stay FP64; cmg_apply,
 * cmg_colour_step, cmg_smooth, cmg_transfer, cmg_coarse_solve and cmg_vcycle
 * convert their FP64 arguments and run in the selected precision. */
cmg_status cmg_set_precision(cmg_problem* p, int fp32);

/* Launch shapes chosen by launch size: cut colour steps of fewer than
 * small_cut_launch patches run with twice the threads per patch block
 * (default 1536; 0 never, a large value always), and the grid-stride operator
 * and interior-patch kernels launch at most max_blocks blocks per column
 * (default 2048, >= 1).  The arithmetic of every node is the same in every
 * configuration, so results are bitwise independent of these choices; tests
 * use it to run the configurations of large levels on small ones.  Host only. */
cmg_status cmg_set_launch(cmg_problem* p, int small_cut_launch, int max_blocks);

/* Ghost-penalty coupling in the residuals of the cut colour steps (paper
 * Section 2.3, last paragraph: the parallel smoother ignores the coupling
 * through ghost penalties between neighbouring vertex patches).
 * mode 0 (default): every patch of a colour solves with the exact residual
 *   (b - A x)[I_j], ghost faces on the patch boundary included; only the
 *   ghost coupling between same-coloured patches, which update at once, is
 *   ignored.  The V-cycle is symmetric (CG applies).
 * mode 1: patch-local residual: x beyond the patch closure (the cell layer
 *   across a ghost face on the patch boundary) counts as zero, i.e. row i of
 *   the residual is b_i - sum_{j in closure} A_ij x_j.  A patch then reads
 *   nothing that a same-coloured patch writes, but a smoothing step no longer
 *   keeps the exact solution fixed and the V-cycle is not symmetric: for
 *   cmg_gmres, cmg_vcycle_solve, cmg_vcycle and the single-level calls only;
 *   cmg_solve and the multi-column calls return CMG_EINVAL while it is set.
 * Host only; takes effect for the following launches. */
cmg_status cmg_set_ghost_coupling(cmg_problem* p, int mode);

/* V-cycles (cmg_vcycle, cmg_vcycle_multi and those inside the solvers) run
 * as replays of HIP graphs: the kernel sequence of a V-cycle is captured once
 * per precision and column count (on a stream of the problem's own) and each
 * V-cycle is one graph launch on the caller's stream, so the host does not
 * issue ~270 kernel launches per V-cycle.  The graphs hold kernel nodes only
 * (no memset nodes); while kernels are timed (cmg_timing), every timed launch
 * is a graph of its own, launched between two events recorded on the stream.
 * Results are bit for bit those of kernel-by-kernel launches.  enable = 0 launches kernel by
 * kernel (default 1).  cmg_set_launch, cmg_set_ghost_coupling, cmg_timing
 * and this call drop the captured graphs.  Host only. */
cmg_status cmg_set_graphs(cmg_problem* p, int enable);

/* Number of DoFs on a level (0 = coarsest, n_levels-1 = finest). */
cmg_status cmg_ndofs(const cmg_problem* p, int level, int64_t* n);

/* y = A_l x on one level (paper eq. (cutfem-ghost) in matrix form). */
cmg_status cmg_apply(cmg_problem* p, int level, const double* x, double* y, void* stream);

/* y = A_l x like cmg_apply, for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no hipMalloc, hipFree or other allocating call, and no kernel
 * timers.  Its intermediates (the level's lattice vectors of x and A x, the
 * ghost-face jumps and the special-cell products) live in one file-scope
 * device array of 32 MiB per device (CMG_NOALLOC_SCRATCH_BYTES), held until
 * the process ends; its device address is taken once per device when a
 * problem is set up or uploaded there.  A level whose intermediates exceed it
 * returns CMG_EINVAL (nothing launched); so does a call from another device
 * than the problem's.  Every call on a GPU uses that GPU's one array: calls
 * that overlap in time on one GPU (other streams, other problems, other
 * threads) race and must be serialised by the caller.  Results equal
 * cmg_apply's bit for bit (same kernels). */
#define CMG_NOALLOC_SCRATCH_BYTES (32u << 20)
cmg_status cmg_apply_noalloc(cmg_problem* p, int level, const double* x, double* y, void* stream);

/* One colour step of the smoother on level >= 1 (paper eq. (local-solver)):
 * for all patches j of the given class (interior != 0: interior patches with
 * fast diagonalisation; 0: cut patches with dense inverses) and colour
 * (0..2^dim-1): x[I_j] += A_j^{-1} (b - A_l x)[I_j], all from the x at entry.
 * x is updated in place. */
cmg_status cmg_colour_step(cmg_problem* p, int level, int interior, int colour, double* x, const double* b,
                           void* stream);

/* One smoothing step S(x, b) on level >= 1: interior colours 0..C-1, then n_c
 * times the cut colours 0..C-1 (eq. (smoother-split)); post != 0 runs the same
 * colour steps in reverse order.  x is updated in place. */
cmg_status cmg_smooth(cmg_problem* p, int level, int post, double* x, const double* b, void* stream);

/* Transfers between level l-1 and l >= 1 (paper Section 2.2): dir = 0
 * prolongation (embedding) y_l = P_l x_{l-1}; dir = 1 restriction y_{l-1} =
 * P_l^T x_l. */
cmg_status cmg_transfer(cmg_problem* p, int level, int dir, const double* x, double* y, void* stream);

/* Exact coarse solve x_0 = A_0^{-1} b_0 on level 0 (paper Section 2.2: the
 * V-cycle ends in an exact solve on the coarsest level; the paper names no
 * solver, here a GEMV with the dense inverse from cmg_setup, FP32 in the
 * mixed-precision mode). */
cmg_status cmg_coarse_solve(cmg_problem* p, const double* b, double* x, void* stream);

/* One V-cycle on the finest level with zero initial guess: z = B r (paper
 * Section 2.2, the standard V-cycle with one pre- and one post-smoothing step
 * of the smoother of eq. (smoother-split); Section 4 for the one-step setting).
 * The post-smoother runs the pre-smoother's colour steps in reverse, so B is
 * symmetric and usable in CG. */
cmg_status cmg_vcycle(cmg_problem* p, const double* r, double* z, void* stream);

/* Solve A_L x = b (paper Section 2.1, eq. (weak-equation) in matrix form) by
 * CG preconditioned with the V-cycle (the paper uses the V-cycle inside
 * GMRES, Section 2.2; the benchmark configurations use CG, which the symmetric
 * V-cycle allows), from x = 0 until ||b - A x||_2 <= rtol ||b||_2, FP64 Krylov
 * vectors and operator products.  Synchronises the stream once per iteration.
 * info may be NULL.  CMG_ENOTCONV after maxit (x holds the last iterate),
 * CMG_EBREAKDOWN when p^T A p <= 0 or is not finite. */
cmg_status cmg_solve(cmg_problem* p, const double* b, double* x, double rtol, int maxit, cmg_solve_info* info,
                     void* stream);

/* The paper's other outer solvers (Section 2.2 and Section 4, its Tables 1-3),
 * from x = 0, with the V-cycle of the current precision as preconditioner and
 * FP64 operator products:
 * cmg_gmres: right-preconditioned restarted GMRES(restart), 1 <= restart < 64;
 *   Arnoldi on A B with classical Gram-Schmidt applied twice; x = B V y.  Stops
 *   when the GMRES residual norm (||b - A x|| in exact arithmetic) is <= rtol
 *   ||b||; info->iterations counts Arnoldi steps (V-cycles).
 * cmg_vcycle_solve: multigrid as a stand-alone solver, x_{k+1} = x_k + B (b - A x_k),
 *   until ||b - A x_k|| <= rtol ||b||; CMG_ENOTCONV once the residual exceeds
 *   1e3 ||b|| (divergence) or after maxit cycles.
 * Both synchronise the stream a few times per iteration; info may be NULL. */
cmg_status cmg_gmres(cmg_problem* p, const double* b, double* x, double rtol, int maxit, int restart,
                     cmg_solve_info* info, void* stream);
cmg_status cmg_vcycle_solve(cmg_problem* p, const double* b, double* x, double rtol, int maxit, cmg_solve_info* info,
                            void* stream);

/* Several right-hand sides at once (1 <= nrhs <= 8).  Column c of r, z, b and x
 * starts at c * n_L (n_L = cmg_ndofs of the finest level), canonical order.
 *
 * cmg_vcycle_multi: z_c = B r_c for every column.  In FP64 the columns run
 * through the same kernels as cmg_vcycle (one grid row per column) and the
 * results equal nrhs single V-cycles bit for bit.  In FP32 (cmg_set_precision)
 * the cut-patch local solves read each inverse once for all columns and apply
 * it on the matrix cores (16x16x4 FP32 MFMA, FP32 accumulation), also for
 * nrhs = 1, so the result differs from cmg_vcycle by rounding only.  In both
 * precisions a column's result is independent of the other columns and of
 * nrhs, bit for bit.
 *
 * cmg_solve_multi: nrhs independent PCG recurrences (own alpha, beta and
 * stopping test per column) that share one multi-column V-cycle and one
 * multi-column FP64 operator product per iteration; a converged column is
 * frozen (alpha = 0) while the others continue.  info (nrhs entries, may be
 * NULL) holds each column's iterations and final relative residual.  Returns
 * CMG_ENOTCONV if any column misses rtol within maxit.
 *
 * The first call allocates multi-column work vectors (8 columns on every
 * level) and, in FP32, a tiled copy of the cut-patch inverses. */
cmg_status cmg_vcycle_multi(cmg_problem* p, int nrhs, const double* r, double* z, void* stream);
cmg_status cmg_solve_multi(cmg_problem* p, int nrhs, const double* b, double* x, double rtol, int maxit,
                           cmg_solve_info* info, void* stream);

/* Grouped V-cycles of several problems (the V-cycle of Section 2.2 for each).
 * For callers that solve many small problems at once, such as a solve server
 * (the V-cycle of a small problem is bound by its ~270 kernel launches, not by
 * memory traffic).  A group holds 1..8 distinct uploaded problems with the same
 * dimension, degree, level count, coarse mesh, box, V-cycle precision and
 * device, all with the exact ghost coupling: their levels share one lattice.
 * cmg_group_create records every member's V-cycle in the form that
 * cmg_vcycle_multi runs with nrhs = 1 (allocating its multi-column vectors as
 * that call does) and checks that the members' kernel sequences match step by
 * step, which holds when every member has cut patches in the same colours on
 * every level; otherwise it returns CMG_EINVAL and keeps nothing.  It uploads
 * the members' kernel arguments as one device table.  Each step of the
 * group's V-cycle is then one launch over all members (blockIdx.z selects the
 * member), and the grouped V-cycle is replayed from one HIP graph.  The group
 * keeps the precision and ghost coupling its members had when it was created.
 * A member stays usable alone, but no other call may run on a member while a
 * call of its group runs, and a group must be destroyed before any of its
 * members.
 *
 * cmg_group_vcycle: z[m] = B_m r[m] for every member m (n_L of that member
 * entries each, canonical order); bit for bit what
 * cmg_vcycle_multi(member, 1, r[m], z[m]) returns.
 * cmg_group_solve: one PCG per member whose V-cycles run grouped; x[m], info[m]
 * and status[m] (info and status may be NULL) are bit for bit those of
 * cmg_solve_multi(member, 1, b[m], x[m], rtol, maxit) (for a breakdown or a
 * non-finite b: that call's status, with x[m] as it left it).  A member that
 * converged or failed is frozen while the others continue.  Returns CMG_OK
 * when every member converged, else the status of the first member that did
 * not. */
typedef struct cmg_group cmg_group;
cmg_status cmg_group_create(cmg_problem* const* members, int n, cmg_group** out);
cmg_status cmg_group_vcycle(cmg_group* g, const double* const* r, double* const* z, void* stream);
cmg_status cmg_group_solve(cmg_group* g, const double* const* b, double* const* x, double rtol, int maxit,
                           cmg_solve_info* info, cmg_status* status, void* stream);
void cmg_group_destroy(cmg_group* g);

/* Kernel timing for measurements.  While kind_mask is non-zero, every kernel
 * launch of a kind whose bit is set is bracketed by HIP events on its stream.
 * Kinds: 0 operator apply / residual, 1 interior colour step, 2 cut colour
 * step (residual + dense solve), 3 cut colour update, 4 prolongation,
 * 5 restriction, 6 coarse solve, 7 layout (zero / scatter / gather),
 * 8 CG vector operations (bits 0..15).  Bits 16..23, when non-zero, hold
 * 1 + the one level whose launches are timed (CMG_EINVAL beyond the
 * finest); zero times every level.  cmg_timing synchronises the device,
 * clears the records and creates the events up front; 0 switches timing
 * off. */
cmg_status cmg_timing(cmg_problem* p, unsigned kind_mask);

/* Launch count and summed event time (ms) of one kernel kind since the last
 * cmg_timing call, on one level (or all levels for level = -1).  Synchronises
 * on the recorded events. */
cmg_status cmg_timing_read(cmg_problem* p, int kind, int level, int64_t* launches, double* total_ms);

/* Load vector of the manufactured problem u = prod_j sin(pi x_j), f = -Laplace u,
 * Dirichlet data g = u (symmetric Nitsche terms), finest level, written to a
 * HOST array of cmg_ndofs(finest) doubles. */
cmg_status cmg_rhs_manufactured(const cmg_problem* p, double* b_host);

/* Load vector of f(x) = sum_q amp[q] cos(pi kappa_q . x + phase[q]) with
 * homogeneous Dirichlet data (g = 0), finest level, HOST output of
 * cmg_ndofs(finest) doubles; kappa holds n_modes * dim integers. */
cmg_status cmg_rhs_fourier(const cmg_problem* p, int n_modes, const int* kappa, const double* amp,
                           const double* phase, double* b_host);

/* The load vector of cmg_rhs_fourier (f = sum_q amp[q] cos(pi kappa_q . x +
 * phase[q]), g = 0, paper eq. (weak-equation)) assembled on the device into
 * b (device pointer, cmg_ndofs(finest) doubles, canonical order), stream
 * ordered.  Same quadrature as the host assembly: tensor Gauss with k+3 points
 * per direction on uncut cells, the columns of the cut-cell rule with quad_n
 * points per smooth piece on cut cells.  Cell vectors are summed in a fixed
 * order, so b is the same bit for bit in every call and on every stream; it
 * differs from the host assembly by rounding only.  kappa, amp and phase are
 * host arrays (n_modes <= 32, quad_n <= 16).  The first call on a problem
 * builds the cut cells' quadrature columns on the host and uploads them
 * (synchronous, allocates; accounted by cmg_device_bytes flag bit 2). */
cmg_status cmg_rhs_fourier_device(cmg_problem* p, int n_modes, const int* kappa, const double* amp,
                                  const double* phase, double* b, void* stream);

/* Host-side description of a level for tests and diagnostics.
 * what = 0: counts, 8 int64 into buf: n_dofs, n_cells_active, n_cut_cells,
 *           n_interior_patches, n_cut_patches, sum of N_j^2 over cut patches,
 *           n_ghost_faces, lattice nodes per direction;
 * what = 1 (CMG_EXPORT_PERM): lattice node index of every DoF (int32,
 *           n_dofs): the permutation from the canonical order of the ABI
 *           vectors to the lattice order the kernels work in (the canonical
 *           order is the ascending lattice order of the active nodes);
 * what = 2: cell flags (uint8 per background cell, bit 0 active, bit 1 cut);
 * what = 3: element matrices of the cut cells in the order of their cell
 *           index, (k+1)^d x (k+1)^d row-major each, cell-local nodes x fastest;
 * what = 4: dense inverse of A_0 (level 0 only), row-major;
 * what = 5 (CMG_EXPORT_QUADRATURE): the cut-cell rule of the element
 *           matrices, double array: per cut cell in cut-id order the column
 *           count m, then m columns of 7 + 2 dim doubles each: height
 *           direction e, base point (dim entries, entry e unused), base
 *           weight w, inside interval [t0, t1] along e (t1 <= t0: none),
 *           surface flag, crossing point t_s, surface weight w_s and outward
 *           unit normal (dim entries).  The volume rule integrates exactly
 *           along every column; int_{T cap Omega} g = sum w int_{t0}^{t1} g
 *           and int_{Gamma cap T} g = sum w_s g(x_s) over the surface columns;
 * what = 16+c: vertex index of every interior patch of colour c (int32;
 *           vertex V has index V_0 + (N+1) V_1 [+ (N+1)^2 V_2]);
 * what = 24+c / 32+c / 40+c / 48+c: cut patches of colour c - node offsets
 *           (int32, n_patch + 1), lattice nodes of their internal DoFs (int32),
 *           dense inverses (double, N_j x N_j each, consecutive), vertex
 *           index (int32, n_patch);
 * what = 56+c: per internal DoF of the cut patches of colour c (order of 32+c),
 *           uint8: bit 0 set if it is also an internal DoF of a cut patch of
 *           the next colour (cyclically) that has cut patches, bit 1 of the
 *           previous one (the copy rule of the two-buffer cut steps);
 * what = 64: the cut region, the active lattice nodes that a cut colour step
 *           reads (int32, ascending).
 * *needed receives the byte size; buf may be NULL to query it. */
cmg_status cmg_export(const cmg_problem* p, int level, int what, void* buf, size_t bytes, size_t* needed);

#define CMG_EXPORT_PERM 1
#define CMG_EXPORT_QUADRATURE 5

void cmg_destroy(cmg_problem* p);

/* ---- serving: continuous batching of solves on one GPU -------------------
 * A server owns max_slots worker threads, each with its own HIP stream.
 * Requests are taken in arrival order.  A free slot takes the oldest queued
 * request together with up to 7 further queued requests of the same geometry,
 * parameters, rtol and maxit, and solves them as one batch: one multi-column
 * PCG (cmg_solve_multi), so the V-cycles of the batch share every kernel
 * launch.  A hierarchy stays resident between batches (least-recently-used idle
 * hierarchies are evicted when a new one needs room); a new hierarchy is
 * admitted when its exact footprint (cmg_footprint with the multi-column
 * buffers, plus the batch's b and x columns), computed before its set-up,
 * fits into hbm_budget_bytes; one that exceeds the whole budget finishes with
 * status CMG_ENOMEM without being set up.  Batches of different slots
 * overlap on the device.  A batch of one request is joined by the only queued
 * requests of other resident, idle geometries of the same lattice shape
 * (dimension, degree, levels, coarse mesh, box, precision, rtol, maxit), up to
 * 8 problems, and solved by one grouped PCG (cmg_group_solve); a group stays
 * cached while its members are resident.  Every result is independent of what
 * else runs and of the batch or group it was solved in, bit for bit (the
 * column arithmetic of cmg_solve_multi does not depend on the other columns,
 * and a grouped solve equals each member's one-column solve).  Intended for callers
 * that submit many solves of differing geometries, degrees and depths. */
typedef struct cmg_server cmg_server;

typedef struct {
  cmg_levelset levelset;   /* copied at submission */
  cmg_params params;
  int n_modes;             /* 0: manufactured right-hand side; else Fourier f (cmg_rhs_fourier), g = 0 */
  const int* kappa;        /* n_modes * dim */
  const double* amp;
  const double* phase;
  double rtol;
  int maxit;
} cmg_request;

typedef struct {
  int status;              /* cmg_status of the request */
  int64_t n_dofs;
  cmg_solve_info info;
  int cache_hit;           /* 1 when the hierarchy was already resident */
  double t_submit, t_start, t_admitted, t_solve_start, t_done;  /* seconds since server creation */
  int batch;               /* number of requests solved together with this one (itself included) */
  int group;               /* problems whose V-cycles ran grouped with this one's (itself included); 1: none */
} cmg_result;

cmg_status cmg_server_create(size_t hbm_budget_bytes, int max_slots, cmg_server** out);
/* Non-blocking; the request is copied. */
cmg_status cmg_submit(cmg_server* s, const cmg_request* req, uint64_t* ticket);
/* CMG_PENDING until the request finished; then fills res, copies the solution
 * (finest level, canonical order) to x_host when given (x_len must equal
 * res->n_dofs) and forgets the request. */
cmg_status cmg_poll(cmg_server* s, uint64_t ticket, cmg_result* res, double* x_host, int64_t x_len);
/* Finishes the queued requests, then releases everything. */
void cmg_server_destroy(cmg_server* s);

/* Message of the last failing call in this thread ("" if none). */
const char* cmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CUTMG_H */
