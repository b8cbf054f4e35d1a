// HIP kernels of the CutFEM vertex-patch multigrid for gfx950 (MI355X).
//
// Data layout: every level keeps its vectors on the full (kN+1)^d node lattice,
// x fastest, with exact zeros at inactive nodes.  Lattice indexing needs no DoF
// index lists inside the patch kernels, and the patches of one colour read
// neighbouring x-rows, which keeps the HBM streams coalesced.  Compact vectors
// (canonical DoF order) exist only at the library boundary.
//
// Operator (paper eq. (cutfem_nitsche) + eq. (cutfem-ghost)), evaluated row by
// row for a node i:
//   (A x)_i = sum_{active cells T containing i} row_i(E_T) x_T
//           + sum_{ghost faces F of those cells} row_i(G_F) x_{T1 u T2}
// with E_T the uncut stiffness (shared, kept in LDS) or the dense matrix of a
// cut cell, and G_F = sum_m c_m (d^m-jump) x (1-D mass on the face) built from
// 1-D tables: a face needs no stored data.  The operator kernel takes the
// terms of the special cells (cut, or with a ghost face) from two pre-passes:
// the mass-contracted jumps of every ghost face, then one value per special
// cell and node.
//
// Smoother colour steps (paper eqs. (local-solver), (smoother-split)):
//   interior patches: one fused kernel - x on the patch closure is staged in
//     LDS, the residual on the (2k-1)^d internal nodes uses the Cartesian
//     stiffness, the local solve is fast diagonalisation (S (x) S (x) S) D^-1
//     (S^T (x) S^T (x) S^T), and the internal values are updated in place.  Same
//     coloured interior patches read only their own closure, so the fused
//     update is race free.
//   cut patches: residual (general rows incl. ghost faces, which may reach into
//     a same-coloured neighbour) and dense inverse GEMV; every patch of the
//     colour must see the state at the start of the step, so the steps of a
//     smoothing pass alternate between two x buffers (read one, write x + d
//     and the previous colour's DoFs into the other), or, for the matrix-core
//     kernel, write the corrections to a buffer that a second kernel adds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "kernels.h"

namespace cmg {
namespace dev {

template <int B, int E>
struct Pow { static constexpr int v = B * Pow<B, E - 1>::v; };
template <int B>
struct Pow<B, 0> { static constexpr int v = 1; };

template <int D, int K>
struct Shape {
  static constexpr int N1 = K + 1;                 // nodes per cell and direction
  static constexpr int NL = Pow<N1, D>::v;         // nodes per cell
  static constexpr int NP1 = 2 * K - 1;            // internal patch nodes per direction
  static constexpr int NP = Pow<NP1, D>::v;        // internal patch nodes
  static constexpr int NC1 = 2 * K + 1;            // patch closure nodes per direction
  static constexpr int NC = Pow<NC1, D>::v;
  static constexpr int PPB = 256 / NP;             // patches per 256-thread block
  // table layout (doubles), see LevelTables on the host
  static constexpr int T_KCELL = 0;
  static constexpr int T_MHAT = T_KCELL + NL * NL;
  static constexpr int T_D0 = T_MHAT + N1 * N1;
  static constexpr int T_D1 = T_D0 + K * N1;
  static constexpr int T_GC = T_D1 + K * N1;
  static constexpr int T_FDS = T_GC + K;
  static constexpr int T_FDD = T_FDS + NP1 * NP1;
  static constexpr int T_P1D = T_FDD + NP;
  static constexpr int T_K1S = T_P1D + NC1 * N1;
  static constexpr int T_SIZE = T_K1S + N1 * N1;
};

// Work index of block b out of n such that the blocks of one XCD take one
// contiguous range of work items.  The chip dispatches workgroups to its 8
// XCDs round-robin by block index and every XCD has its own L2, so without
// the remap consecutive (spatially neighbouring) cut patches land on
// different XCDs and each XCD fetches the x-lines they share separately
// (measured: finest cut steps 2.5% faster in FP64 and FP32).  The grid-stride
// operator and interior-patch kernels keep the plain order, which measured
// faster for them (the remap cost them 8% and 20%).
// Bijective on [0, n): XCD x < n % 8 takes n / 8 + 1 items, the others n / 8.
__device__ __forceinline__ int xcd_block(int b, int n) {
  constexpr int NX = 8;
  const int q = n / NX, r = n % NX, xc = b % NX, s = b / NX;
  return xc < r ? xc * (q + 1) + s : r * (q + 1) + (xc - r) * q + s;
}

// Grouped launch: one launch runs the same kernel for several problems, the
// problem's argument record being entry blockIdx.z of a device table.  The
// grid is the largest of the members' grids, so every kernel with a grouped
// form lets the blocks beyond its own work return (grid-stride loops, index
// bounds, or a patch index past the colour's patches).
template <int LB, typename A>
__global__ __launch_bounds__(LB) void k_grouped(const A* __restrict__ tab) {
  tab[blockIdx.z].run();
}

__device__ __forceinline__ int64_t lat(int D, int nn, const int* I) {
  return D == 2 ? I[0] + (int64_t)nn * I[1] : I[0] + (int64_t)nn * (I[1] + (int64_t)nn * I[2]);
}

__device__ __forceinline__ int64_t cell_lin(int D, int N, const int* c) {
  return D == 2 ? c[0] + (int64_t)N * c[1] : c[0] + (int64_t)N * (c[1] + (int64_t)N * c[2]);
}

template <int D, int K>
__device__ void load_tables(const double* __restrict__ g, double* s, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = g[i];
}

// Ghost-face pre-pass of the operator: for every ghost face and derivative order
// m, the jump J_m(b_t) = sum_bd psi_bd^(m)(1) x_lower - psi_bd^(m)(0) x_upper at the
// tangential face nodes b_t, contracted with the reference face mass:
// W_m(i_t) = sum_{b_t} prod_j Mhat[i_t,j, b_t,j] J_m(b_t).  A row of a node i of
// a cell adjacent to the face then only needs gc_m * trace_m(i_dir) * W_m(i_t).
// One thread per face and column: the 2 (k+1) nodes along the normal at each
// tangential node are read once for all k orders.
template <int D, int K, typename T>
__device__ __forceinline__ void face_w_body(KLevel L, const T* __restrict__ x, T* __restrict__ W) {
  using S = Shape<D, K>;
  constexpr int N1 = S::N1;
  constexpr int NT = Pow<N1, D - 1>::v;
  x += blockIdx.y * L.n_nodes;  // column blockIdx.y
  W += blockIdx.y * L.n_faces * K * NT;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= L.n_faces) return;
  const double* mh = L.tables + S::T_MHAT;
  const double* d0 = L.tables + S::T_D0;
  const double* d1 = L.tables + S::T_D1;
  const int dir = L.face_dir[f];
  int c[3];
  {
    int64_t r = L.face_lower[f];
#pragma unroll
    for (int a = 0; a < D; ++a) { c[a] = static_cast<int>(r % L.N); r /= L.N; }
  }
  // first node of the lower cell and the lattice strides
  int64_t base = 0, sn = 1, st0 = 0, st1 = 0;
  {
    int64_t sa = 1;
    int tb = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      base += K * c[a] * sa;
      if (a == dir) sn = sa;
      else if (tb++ == 0) st0 = sa;
      else st1 = sa;
      sa *= L.nn;
    }
  }
  T J[K][NT];
#pragma unroll
  for (int bt = 0; bt < NT; ++bt) {
    const int64_t el = base + (bt % N1) * st0 + (D == 3 ? (bt / N1) * st1 : 0);
    T xl[N1], xu[N1];
#pragma unroll
    for (int bd = 0; bd <= K; ++bd) {
      xl[bd] = x[el + bd * sn];
      xu[bd] = x[el + (bd + K) * sn];
    }
#pragma unroll
    for (int m = 0; m < K; ++m) {
      T acc = 0;
#pragma unroll
      for (int bd = 0; bd <= K; ++bd) acc += (T)d1[m * N1 + bd] * xl[bd] - (T)d0[m * N1 + bd] * xu[bd];
      J[m][bt] = acc;
    }
  }
#pragma unroll
  for (int m = 0; m < K; ++m) {
    T* out = W + (f * K + m) * NT;
    if (D == 2) {
#pragma unroll
      for (int it = 0; it < N1; ++it) {
        T acc = 0;
#pragma unroll
        for (int bt = 0; bt < N1; ++bt) acc += (T)mh[it * N1 + bt] * J[m][bt];
        out[it] = acc;
      }
      continue;
    }
    T H[NT];  // (Mhat x Mhat) J by two 1-D contractions
#pragma unroll
    for (int b1 = 0; b1 < N1; ++b1)
#pragma unroll
      for (int i0 = 0; i0 < N1; ++i0) {
        T acc = 0;
#pragma unroll
        for (int b0 = 0; b0 < N1; ++b0) acc += (T)mh[i0 * N1 + b0] * J[m][b0 + N1 * b1];
        H[i0 + N1 * b1] = acc;
      }
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1)
#pragma unroll
      for (int i0 = 0; i0 < N1; ++i0) {
        T acc = 0;
#pragma unroll
        for (int b1 = 0; b1 < N1; ++b1) acc += (T)mh[i1 * N1 + b1] * H[i0 + N1 * b1];
        out[i0 + N1 * i1] = acc;
      }
  }
}

template <int D, int K, typename T>
__global__ __launch_bounds__(256) void k_face_w(KLevel L, const T* __restrict__ x, T* __restrict__ W) {
  face_w_body<D, K, T>(L, x, W);
}

// argument record of k_face_w for grouped launches (k_grouped)
template <int D, int K, typename T>
struct FaceWArgs {
  KLevel L;
  const T* x;
  T* W;
  __device__ void run() const { face_w_body<D, K, T>(L, x, W); }
};

// Special-cell pre-pass of the operator.  A special cell T is cut or has a
// ghost face; for each of them and every column it forms the contribution of T
// to the rows of its nodes,
//   C_T(i) = (E_T x_T)_i + sum_{ghost faces F of T} sum_m gc_m trace_m(i_dir) W_m(F)(i_t),
// with E_T the cut-cell matrix or the uncut stiffness and W the face pre-pass
// output, so that the operator kernel adds one value per special cell and
// node.  CPB cells per 64-thread block, one thread per cell node, the columns
// together.  A cut cell's E_T is symmetric and read as its packed upper
// triangle, (k+1)^d ((k+1)^d + 1) / 2 entries instead of (k+1)^{2d}, staged in
// LDS by the cell's threads (consecutive threads, consecutive entries).
template <int D, int K>
struct CellShape {
  static constexpr int NL = Shape<D, K>::NL;
  static constexpr int CPB = 64 / NL;
  static_assert(CPB >= 1, "one thread per cell node");
};

template <int D, int K, typename T, int NCOL>
__device__ __forceinline__ void cell_ax_body(KLevel L, const T* __restrict__ x, const T* __restrict__ W,
                                             T* __restrict__ C, int ncol) {
  using S = Shape<D, K>;
  constexpr int N1 = S::N1, NL = S::NL, CPB = CellShape<D, K>::CPB, NF = 2 * D;
  constexpr int NT = Pow<N1, D - 1>::v;
  constexpr int NPK = NL * (NL + 1) / 2;  // entries of a packed symmetric cell matrix
  __shared__ T xs[CPB][NL][NCOL];
  __shared__ T epk[CPB][NPK];
  const int lc = threadIdx.x / NL;
  const int i = threadIdx.x % NL;
  const int64_t t = (int64_t)blockIdx.x * CPB + lc;
  const bool on = lc < CPB && t < L.n_spec;
  int il[3] = {0, 0, 0};
  int32_t info[1 + NF];
  if (on) {
    int64_t r = L.spec_cells[t];
#pragma unroll
    for (int j = 0; j <= NF; ++j) info[j] = L.spec_info[t * (1 + NF) + j];
    int I[3];
    int q = i;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      il[a] = q % N1;
      q /= N1;
      I[a] = K * static_cast<int>(r % L.N) + il[a];
      r /= L.N;
    }
    const int64_t node = lat(D, L.nn, I);
#pragma unroll
    for (int c = 0; c < NCOL; ++c) xs[lc][i][c] = c < ncol ? x[c * L.n_nodes + node] : (T)0;
    // a cut cell's matrix, read once as its packed upper triangle (the cell's
    // threads read consecutive entries, G loads in flight per thread) and
    // staged for all rows
    if (info[0] >= 0) {
      const T* P = L.cut_packed_t<T>() + (int64_t)info[0] * NPK;
      constexpr int NR = (NPK + NL - 1) / NL, G = 8;
#pragma unroll
      for (int r0 = 0; r0 < NR; r0 += G) {
        T v[G];
#pragma unroll
        for (int r = 0; r < G; ++r) {
          const int e = (r0 + r) * NL + i;
          v[r] = (r0 + r < NR && e < NPK) ? P[e] : (T)0;
        }
#pragma unroll
        for (int r = 0; r < G; ++r) {
          const int e = (r0 + r) * NL + i;
          if (r0 + r < NR && e < NPK) epk[lc][e] = v[r];
        }
      }
    }
  }
  __syncthreads();
  if (!on) return;
  T acc[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) acc[c] = 0;
  // ghost terms first: their loads do not wait for the staged x
  const int64_t wcol = L.n_faces * K * NT;
  const double* d0 = L.tables + S::T_D0;
  const double* d1 = L.tables + S::T_D1;
  const double* gc = L.tables + S::T_GC;
#pragma unroll
  for (int dir = 0; dir < D; ++dir) {
    int it = 0, st = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (a == dir) continue;
      it += il[a] * st;
      st *= N1;
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int fid = info[1 + 2 * dir + side];
      if (fid < 0) continue;
      const T* w = W + (int64_t)fid * K * NT + it;
#pragma unroll
      for (int m = 0; m < K; ++m) {
        const T sg = (T)(gc[m] * (side == 1 ? d1[m * N1 + il[dir]] : -d0[m * N1 + il[dir]]));
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
          if (c < ncol) acc[c] += sg * w[c * wcol + m * NT];
      }
    }
  }
  T cell[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) cell[c] = 0;
  if (info[0] >= 0) {
    // entry (a, b), a <= b, of the packed upper triangle sits at a (2 NL - a + 1) / 2 + b - a;
    // row i of E is (j, i) for j < i and (i, j) from the diagonal on
    const int rowi = i * (2 * NL - i + 1) / 2;
#pragma unroll 4
    for (int j = 0; j < NL; ++j) {
      const int q = j < i ? j * (2 * NL - j + 1) / 2 + (i - j) : rowi + (j - i);
      const T e = epk[lc][q];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) cell[c] += e * xs[lc][j][c];
    }
  } else {
    const T* row = L.kcell_t<T>() + S::T_KCELL + i * NL;
#pragma unroll 4
    for (int j = 0; j < NL; ++j) {
      const T e = row[j];
#pragma unroll
      for (int c = 0; c < NCOL; ++c) cell[c] += e * xs[lc][j][c];
    }
  }
#pragma unroll
  for (int c = 0; c < NCOL; ++c)
    if (c < ncol) C[c * L.n_spec * NL + t * NL + i] = cell[c] + acc[c];
}

template <int D, int K, typename T, int NCOL>
__global__ __launch_bounds__(64) void k_cell_ax(KLevel L, const T* __restrict__ x, const T* __restrict__ W,
                                                T* __restrict__ C, int ncol) {
  cell_ax_body<D, K, T, NCOL>(L, x, W, C, ncol);
}

// argument record of k_cell_ax for grouped launches (k_grouped)
template <int D, int K, typename T, int NCOL>
struct CellAxArgs {
  KLevel L;
  const T* x;
  const T* W;
  T* C;
  int ncol;
  __device__ void run() const { cell_ax_body<D, K, T, NCOL>(L, x, W, C, ncol); }
};

template <int D, int K>
struct ApplyShape {
  static constexpr int B = (D == 3 && K == 3) ? 2 : 4;   // cells per tile and direction
  static constexpr int R1 = (B + 1) * K + 1;             // staged nodes per direction: cells -1 .. B-1
  static constexpr int NR = Pow<R1, D>::v;
  static constexpr int C1 = B + 1;                       // staged cells per direction
  static constexpr int NCC = Pow<C1, D>::v;
  static constexpr int O1 = B * K + 1;                   // owned nodes per direction (last tile: + 1)
  static constexpr int NO = Pow<O1, D>::v;
};

// y = A x (b == nullptr) or y = b - A x on the active nodes of a tile of B^d
// cells.  x on the cells -1 .. B-1 around the tile is staged in LDS; every
// owned node sums, over the cells that contain it, the uncut stiffness row
// (from LDS) or the special-cell value of the pre-pass (from C).  The C loads
// of a node's cells are independent and issued together before the LDS rows.
template <int D, int K, typename T>
__device__ __forceinline__ void apply_body(KLevel L, const T* __restrict__ x, const T* __restrict__ b,
                                           T* __restrict__ y, const T* __restrict__ C) {
  using S = Shape<D, K>;
  using A = ApplyShape<D, K>;
  constexpr int N1 = S::N1, NL = S::NL, B = A::B, R1 = A::R1, C1 = A::C1, O1 = A::O1;
  constexpr int NCB = 1 << D;
  constexpr int NRW = N1 * (D == 3 ? N1 : 1);
  __shared__ T tab[S::T_MHAT];  // uncut stiffness, in the path's precision
  __shared__ T xs[A::NR];
  __shared__ int32_t csid[A::NCC];
  for (int i = threadIdx.x; i < S::T_MHAT; i += blockDim.x) tab[i] = L.kcell_t<T>()[i];
  x += blockIdx.y * L.n_nodes;  // column blockIdx.y
  if (b) b += blockIdx.y * L.n_nodes;
  y += blockIdx.y * L.n_nodes;
  C += blockIdx.y * L.n_spec * NL;
  const int NTd = (L.N + B - 1) / B;
  for (int ti = blockIdx.x; ti < L.n_tiles; ti += gridDim.x) {
    __syncthreads();
    int tc[3] = {0, 0, 0};
    {
      int r = L.tiles[ti];
#pragma unroll
      for (int a = 0; a < D; ++a) { tc[a] = r % NTd; r /= NTd; }
    }
    for (int e = threadIdx.x; e < A::NCC; e += blockDim.x) {
      int c[3];
      bool in = true;
      int r = e;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        c[a] = B * tc[a] - 1 + r % C1;
        r /= C1;
        in = in && c[a] >= 0 && c[a] < L.N;
      }
      csid[e] = in ? L.cell_sid[cell_lin(D, L.N, c)] : -2;
    }
    for (int e = threadIdx.x; e < A::NR; e += blockDim.x) {
      int I[3];
      bool in = true;
      int r = e;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        I[a] = K * (B * tc[a] - 1) + r % R1;
        r /= R1;
        in = in && I[a] >= 0 && I[a] < L.nn;
      }
      xs[e] = in ? x[lat(D, L.nn, I)] : (T)0;
    }
    __syncthreads();
    // the node's cells along each direction: a node on a cell boundary
    // (q % K == 0) lies in staged cells q/K (local index K) and q/K + 1 (local
    // index 0), any other node only in q/K + 1; comb bit a selects the upper one
    auto cell_of = [&](const int* q, int comb, int* c, int* il) {
      bool ok = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int sel = (comb >> a) & 1;
        if (q[a] % K == 0) {
          c[a] = q[a] / K + sel;
          il[a] = sel ? 0 : K;
        } else {
          ok = ok && sel == 0;
          c[a] = q[a] / K + 1;
          il[a] = q[a] % K;
        }
        ok = ok && c[a] < C1;  // beyond the background box
      }
      return ok;
    };
#pragma unroll 1
    for (int e = threadIdx.x; e < A::NO; e += blockDim.x) {
      int q[3], I[3];
      bool own = true;
      int r = e;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        q[a] = r % O1;
        r /= O1;
        I[a] = K * B * tc[a] + q[a];
        // the layer q = B K belongs to the next tile unless this is the last one
        own = own && I[a] < L.nn && (q[a] < B * K || tc[a] == NTd - 1);
      }
      if (!own) continue;
      const int64_t node = lat(D, L.nn, I);
      const T bv = b ? b[node] : (T)0;
      // pass 1: the special-cell values, all loads in flight together
      T cv[NCB];
      bool act = false;  // the node lies in an active cell
#pragma unroll
      for (int comb = 0; comb < NCB; ++comb) {
        cv[comb] = 0;
        int c[3], il[3];
        if (!cell_of(q, comb, c, il)) continue;
        int ce = c[0] + C1 * c[1];
        if (D == 3) ce += C1 * C1 * c[2];
        const int sid = csid[ce];
        if (sid == -2) continue;  // inactive cell
        act = true;
        if (sid < 0) continue;
        int iloc = il[0] + N1 * il[1];
        if (D == 3) iloc += N1 * N1 * il[2];
        cv[comb] = C[(int64_t)sid * NL + iloc];
      }
      if (!act) continue;
      // pass 2: uncut stiffness rows of the regular cells from LDS
      T ax = 0;
#pragma unroll 1
      for (int comb = 0; comb < NCB; ++comb) {
        int c[3], il[3];
        if (!cell_of(q, comb, c, il)) continue;
        int ce = c[0] + C1 * c[1];
        if (D == 3) ce += C1 * C1 * c[2];
        if (csid[ce] != -1) continue;
        int iloc = il[0] + N1 * il[1];
        if (D == 3) iloc += N1 * N1 * il[2];
        int xb = K * c[0] + R1 * K * c[1];
        if (D == 3) xb += R1 * R1 * K * c[2];
        const T* row = tab + iloc * NL;
        T acc[NRW];
#pragma unroll
        for (int a = 0; a < NRW; ++a) acc[a] = 0;
#pragma unroll
        for (int bq = 0; bq < NL; ++bq) {
          const int b0 = bq % N1, b12 = bq / N1;
          const int xi = xb + b0 + R1 * (b12 % N1) + (D == 3 ? R1 * R1 * (b12 / N1) : 0);
          acc[b12] += row[bq] * xs[xi];
        }
        T sacc = 0;
#pragma unroll
        for (int a = 0; a < NRW; ++a) sacc += acc[a];
        ax += sacc;
      }
#pragma unroll
      for (int comb = 0; comb < NCB; ++comb) ax += cv[comb];
      y[node] = b ? bv - ax : ax;
    }
  }
}

template <int D, int K, typename T>
__global__ __launch_bounds__(256) void k_apply(KLevel L, const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, const T* __restrict__ C) {
  apply_body<D, K, T>(L, x, b, y, C);
}

// argument record of k_apply for grouped launches (k_grouped)
template <int D, int K, typename T>
struct ApplyArgs {
  KLevel L;
  const T* x;
  const T* b;
  T* y;
  const T* C;
  __device__ void run() const { apply_body<D, K, T>(L, x, b, y, C); }
};

// Entry (s, j) of the 1-D matrix assembled from the element matrix e ((k+1) x
// (k+1), row-major) over the NCELL staged cells of an operator tile along one
// direction (cell c holds staged nodes K c .. K c + K).  tile1d_nz tells
// whether some cell holds both nodes; with compile-time s and j both fold.
template <int K, int NCELL>
__host__ __device__ constexpr bool tile1d_nz(int s, int j) {
  for (int c = 0; c < NCELL; ++c)
    if (s >= K * c && s <= K * c + K && j >= K * c && j <= K * c + K) return true;
  return false;
}
template <int K, int NCELL>
__device__ __forceinline__ double tile1d(const double* e, int s, int j) {
  double v = 0;
#pragma unroll
  for (int c = 0; c < NCELL; ++c)
    if (s >= K * c && s <= K * c + K && j >= K * c && j <= K * c + K) v += e[(s - K * c) * (K + 1) + (j - K * c)];
  return v;
}
// The same for a run-time row s: the cells holding s are s/K - 1 and s/K when
// s is a cell boundary, else s/K.
template <int K, int NCELL>
__device__ __forceinline__ double tile1d_rt(const double* e, int s, int j) {
  const int c1 = s / K, c0 = s % K == 0 ? c1 - 1 : c1;
  double v = 0;
  for (int c = c0; c <= c1; ++c)
    if (c >= 0 && c < NCELL && j >= K * c && j <= K * c + K) v += e[(s - K * c) * (K + 1) + (j - K * c)];
  return v;
}

// y = A x (b == nullptr) or y = b - A x on the active nodes of a tile whose
// staged cells -1 .. B-1 are all active and regular.  There A is the sum over
// directions a of tensor products of the assembled 1-D stiffness h^(d-2) K1
// along a and the assembled 1-D mass along the others (the uncut cell
// stiffness has this form, summed over the staged cells), applied by one pass
// per direction: along the slowest direction every staged line gives Mhat x
// and Khat x on the owned rows; in 3-D the next direction gives Mhat Mhat x and
// Khat Mhat x + Mhat Khat x; every owned node contracts direction 0 at its own
// position.  Only the band of the 1-D matrices is applied.
template <int D, int K, typename T>
__device__ __forceinline__ void apply_sf_body(KLevel L, const T* __restrict__ x, const T* __restrict__ b,
                                              T* __restrict__ y) {
  using S = Shape<D, K>;
  using A = ApplyShape<D, K>;
  constexpr int N1 = S::N1, B = A::B, R1 = A::R1, C1 = A::C1, O1 = A::O1;
  constexpr int NW = D == 3 ? R1 * O1 * O1 : 1;                      // values per second-pass array
  constexpr int NXV = D == 3 ? (A::NR > 2 * NW ? A::NR : 2 * NW) : A::NR;
  constexpr int NU = D == 3 ? R1 * R1 * O1 : R1 * O1;                // values per first-pass array
  __shared__ double m1[N1 * N1], k1[N1 * N1];
  __shared__ T xv[NXV];     // x staged; in 3-D then the second pass: [0, NW) and [NW, 2 NW)
  __shared__ T ua[2][NU];   // first pass: Mhat x and Khat x along the slowest direction
  for (int i = threadIdx.x; i < N1 * N1; i += blockDim.x) {
    m1[i] = L.tables[S::T_MHAT + i];
    k1[i] = L.tables[S::T_K1S + i];
  }
  x += blockIdx.y * L.n_nodes;  // column blockIdx.y
  if (b) b += blockIdx.y * L.n_nodes;
  y += blockIdx.y * L.n_nodes;
  const int NTd = (L.N + B - 1) / B;
  for (int ti = blockIdx.x; ti < L.n_tiles_sf; ti += gridDim.x) {
    __syncthreads();  // tables, and the previous tile finished with the LDS buffers
    int tc[3] = {0, 0, 0};
    {
      int r = L.tiles_sf[ti];
#pragma unroll
      for (int a = 0; a < D; ++a) { tc[a] = r % NTd; r /= NTd; }
    }
    for (int e = threadIdx.x; e < A::NR; e += blockDim.x) {
      int I[3];
      bool in = true;
      int r = e;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        I[a] = K * (B * tc[a] - 1) + r % R1;
        r /= R1;
        in = in && I[a] >= 0 && I[a] < L.nn;
      }
      xv[e] = in ? x[lat(D, L.nn, I)] : (T)0;
    }
    __syncthreads();
    // slowest direction: every staged line, rows K .. K + O1 - 1
    constexpr int NLA = D == 3 ? R1 * R1 : R1;
    for (int l = threadIdx.x; l < NLA; l += blockDim.x) {
      T xl[R1];
#pragma unroll
      for (int j = 0; j < R1; ++j) xl[j] = xv[l + NLA * j];
#pragma unroll
      for (int q = 0; q < O1; ++q) {
        T um = 0, uk = 0;
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          if (!tile1d_nz<K, C1>(K + q, j)) continue;
          um += (T)tile1d<K, C1>(m1, K + q, j) * xl[j];
          uk += (T)tile1d<K, C1>(k1, K + q, j) * xl[j];
        }
        ua[0][l * O1 + q] = um;
        ua[1][l * O1 + q] = uk;
      }
    }
    __syncthreads();
    if constexpr (D == 3) {
      // direction 1 on the lines (s0, q2): Mhat Mhat x into [0, NW), Khat Mhat x + Mhat Khat x into [NW, 2 NW)
      for (int t = threadIdx.x; t < R1 * O1; t += blockDim.x) {
        const int s0 = t % R1, q2 = t / R1;
        T ul[R1], kl[R1];
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          ul[j] = ua[0][(s0 + R1 * j) * O1 + q2];
          kl[j] = ua[1][(s0 + R1 * j) * O1 + q2];
        }
#pragma unroll
        for (int q = 0; q < O1; ++q) {
          T vmm = 0, vxx = 0;
#pragma unroll
          for (int j = 0; j < R1; ++j) {
            if (!tile1d_nz<K, C1>(K + q, j)) continue;
            vmm += (T)tile1d<K, C1>(m1, K + q, j) * ul[j];
            vxx += (T)tile1d<K, C1>(k1, K + q, j) * ul[j];
            vxx += (T)tile1d<K, C1>(m1, K + q, j) * kl[j];
          }
          xv[s0 + R1 * (q + O1 * q2)] = vmm;
          xv[NW + s0 + R1 * (q + O1 * q2)] = vxx;
        }
      }
      __syncthreads();
    }
    // direction 0 at every owned node: Khat (first array) + Mhat (second array)
    const T* f0 = D == 3 ? xv : &ua[0][0];
    const T* f1 = D == 3 ? xv + NW : &ua[1][0];
#pragma unroll 1
    for (int e = threadIdx.x; e < A::NO; e += blockDim.x) {
      int q[3], I[3];
      bool own = true;
      int r = e;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        q[a] = r % O1;
        r /= O1;
        I[a] = K * B * tc[a] + q[a];
        // the layer q = B K belongs to the next tile unless this is the last one
        own = own && I[a] < L.nn && (q[a] < B * K || tc[a] == NTd - 1);
      }
      if (!own) continue;
      const int64_t node = lat(D, L.nn, I);
      const T bv = b ? b[node] : (T)0;
      const int s = K + q[0];
      // second-pass value of staged column j: 3-D index j + R1 (q1 + O1 q2), 2-D j O1 + q1
      const int rest = D == 3 ? R1 * (q[1] + O1 * q[2]) : q[1];
      T ax = 0;
#pragma unroll
      for (int dj = -K; dj <= K; ++dj) {
        // s >= K, so j >= 0; the line ends at R1 - 1 = (B + 1) K, so for K >= 2
        // the last owned rows reach past it: those j hold no matrix entry, and
        // the words past the line were not written by this block (not
        // necessarily finite), so they are skipped
        const int j = s + dj;
        if (j >= R1) continue;
        const int at = D == 3 ? j + rest : j * O1 + rest;
        ax += (T)tile1d_rt<K, C1>(k1, s, j) * f0[at];
        ax += (T)tile1d_rt<K, C1>(m1, s, j) * f1[at];
      }
      y[node] = b ? bv - ax : ax;
    }
  }
}

template <int D, int K, typename T>
__global__ __launch_bounds__(256) void k_apply_sf(KLevel L, const T* __restrict__ x, const T* __restrict__ b,
                                                  T* __restrict__ y) {
  apply_sf_body<D, K, T>(L, x, b, y);
}

// argument record of k_apply_sf for grouped launches (k_grouped)
template <int D, int K, typename T>
struct ApplySfArgs {
  KLevel L;
  const T* x;
  const T* b;
  T* y;
  __device__ void run() const { apply_sf_body<D, K, T>(L, x, b, y); }
};

// Entry (r, j) of a 1-D matrix assembled on the 2k+1 closure nodes of a patch
// from the element matrix e ((k+1) x (k+1), row-major) of its two cells, the
// second cell starting at node k.  patch1d_nz tells whether some cell holds
// both nodes; with compile-time r and j both fold to constants.
template <int K>
__device__ __forceinline__ constexpr bool patch1d_nz(int r, int j) {
  return (r <= K && j <= K) || (r >= K && j >= K);
}
template <int K, typename E>
__device__ __forceinline__ E patch1d(const E* e, int r, int j) {
  E v = 0;
  if (r <= K && j <= K) v += e[r * (K + 1) + j];
  if (r >= K && j >= K) v += e[(r - K) * (K + 1) + (j - K)];
  return v;
}
// The same with a run-time row r: each term is read when its cell holds both nodes.
template <int K, typename E>
__device__ __forceinline__ E patch1d_rt(const E* e, int r, int j) {
  const E lo = (r <= K && j <= K) ? e[(r <= K ? r : 0) * (K + 1) + (j <= K ? j : 0)] : E(0);
  const E hi = (r >= K && j >= K) ? e[(r >= K ? r - K : 0) * (K + 1) + (j >= K ? j - K : 0)] : E(0);
  return lo + hi;
}

// Fused colour step over interior patches.
template <int D, int K, typename T>
__device__ __forceinline__ void interior_step_body(KLevel L, const int32_t* __restrict__ verts, int nv,
                                                   T* __restrict__ x, const T* __restrict__ b) {
  using S = Shape<D, K>;
  constexpr int NP = S::NP, NP1 = S::NP1, NC = S::NC, NC1 = S::NC1, PPB = S::PPB, N1 = S::N1, NL = S::NL;
  // the level tables this kernel reads, in the precision of the path: 1-D mass,
  // scaled 1-D stiffness, fast-diagonalisation eigenvectors and inverse sums
  __shared__ T cm1[N1 * N1], ck1[N1 * N1], cfs[NP1 * NP1], cfd[NP];
  __shared__ T xs[PPB][NC];
  __shared__ T ra[PPB][NP];
  __shared__ T rb[PPB][NP];
  __shared__ int64_t pbase[PPB];  // lattice index of each patch's closure corner (-1: no patch)
  // sum-factorisation intermediates: after the slowest direction (3-D only) and
  // after the next one, per closure line of the remaining directions
  __shared__ T su[D == 3 ? PPB : 1][D == 3 ? NC1 * NC1 : 1][NP1];
  __shared__ T sk[D == 3 ? PPB : 1][D == 3 ? NC1 * NC1 : 1][NP1];
  __shared__ T vm[PPB][NC1][D == 3 ? NP1 * NP1 : NP1];
  __shared__ T vx[PPB][NC1][D == 3 ? NP1 * NP1 : NP1];
  for (int i = threadIdx.x; i < N1 * N1; i += blockDim.x) {
    cm1[i] = (T)L.tables[S::T_MHAT + i];
    ck1[i] = (T)L.tables[S::T_K1S + i];
  }
  for (int i = threadIdx.x; i < NP1 * NP1; i += blockDim.x) cfs[i] = (T)L.tables[S::T_FDS + i];
  for (int i = threadIdx.x; i < NP; i += blockDim.x) cfd[i] = (T)L.tables[S::T_FDD + i];
  x += blockIdx.y * L.n_nodes;  // column blockIdx.y
  b += blockIdx.y * L.n_nodes;
  const int p = threadIdx.x / NP, i = threadIdx.x % NP;
  const int NV = L.N + 1;
  const int64_t nn = L.nn, nn2 = nn * nn;
  const int ngroups = (nv + PPB - 1) / PPB;
  // lattice offset of the thread's internal node from the closure corner
  int pi[3] = {0, 0, 0};
  int64_t ioff = 0;
  {
    int ri = i;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pi[a] = ri % NP1 + 1;
      ri /= NP1;
    }
    ioff = pi[0] + nn * pi[1] + (D == 3 ? nn2 * pi[2] : 0);
  }
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
  const int gp0 = grp * PPB;
  __syncthreads();  // previous group finished with the LDS buffers
  if (threadIdx.x < PPB) {
    int64_t base = -1;
    if (gp0 + (int)threadIdx.x < nv) {
      int vr = verts[gp0 + threadIdx.x];
      int J[3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        J[a] = K * (vr % NV) - K;
        vr /= NV;
      }
      base = lat(D, L.nn, J);
    }
    pbase[threadIdx.x] = base;
  }
  __syncthreads();
  // stage the closures of all patches of this block: all loads first, then the LDS stores
  {
    constexpr int NST = PPB * NC, NIT = (NST + 255) / 256;
    T v[NIT];
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = threadIdx.x + 256 * u;
      v[u] = 0;
      if (e < NST) {
        const int pp = e / NC, q = e % NC;
        const int64_t base = pbase[pp];
        if (base >= 0) {
          const int q0 = q % NC1, q1 = (q / NC1) % NC1, q2 = q / (NC1 * NC1);
          v[u] = x[base + q0 + nn * q1 + (D == 3 ? nn2 * q2 : 0)];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < NST) xs[e / NC][e % NC] = v[u];
    }
  }
  __syncthreads();
  const bool active = p < PPB && gp0 + p < nv;
  int64_t node = 0;
  T bnode = 0;
  if (active) {
    node = pbase[p] + ioff;
    bnode = b[node];
  }
  // residual b - A x at the internal nodes by sum factorisation on the closure.
  // An interior patch's 2^d cells are all uncut, so A restricted to it is the
  // sum over directions a of tensor products with the assembled 1-D stiffness
  // (h^(d-2) K1) along a and the assembled 1-D mass along the others (each 1-D
  // matrix on the 2k+1 closure nodes is the sum of the two cells' element
  // matrices).  Contractions run from the slowest direction to the fastest;
  // only the internal rows 1..2k-1 of each direction are formed.
  {
    const T* m1 = cm1;
    const T* k1 = ck1;
    if constexpr (D == 3) {
      // direction 2: um = Mhat_2 x, uk = Khat_2 x on every (q0, q1) line
      for (int t = threadIdx.x; t < PPB * NC1 * NC1; t += blockDim.x) {
        const int pp = t / (NC1 * NC1), l = t % (NC1 * NC1);
        if (gp0 + pp >= nv) continue;
        T xv[NC1];
#pragma unroll
        for (int j = 0; j < NC1; ++j) xv[j] = xs[pp][l + NC1 * NC1 * j];
#pragma unroll
        for (int r = 1; r <= NP1; ++r) {
          T um = 0, uk = 0;
#pragma unroll
          for (int j = 0; j < NC1; ++j) {
            if (!patch1d_nz<K>(r, j)) continue;
            um += (T)patch1d<K>(m1, r, j) * xv[j];
            uk += (T)patch1d<K>(k1, r, j) * xv[j];
          }
          su[pp][l][r - 1] = um;
          sk[pp][l][r - 1] = uk;
        }
      }
      __syncthreads();
      // direction 1: vm = Mhat_1 um, vx = Khat_1 um + Mhat_1 uk on every (q0, r2) line
      for (int t = threadIdx.x; t < PPB * NC1 * NP1; t += blockDim.x) {
        const int pp = t / (NC1 * NP1), q0 = (t / NP1) % NC1, r2 = t % NP1;
        if (gp0 + pp >= nv) continue;
        T uv[NC1], kv[NC1];
#pragma unroll
        for (int j = 0; j < NC1; ++j) {
          uv[j] = su[pp][q0 + NC1 * j][r2];
          kv[j] = sk[pp][q0 + NC1 * j][r2];
        }
#pragma unroll
        for (int r = 1; r <= NP1; ++r) {
          T vmv = 0, vxv = 0;
#pragma unroll
          for (int j = 0; j < NC1; ++j) {
            if (!patch1d_nz<K>(r, j)) continue;
            vmv += (T)patch1d<K>(m1, r, j) * uv[j];
            vxv += (T)patch1d<K>(k1, r, j) * uv[j];
            vxv += (T)patch1d<K>(m1, r, j) * kv[j];
          }
          vm[pp][q0][(r - 1) + NP1 * r2] = vmv;
          vx[pp][q0][(r - 1) + NP1 * r2] = vxv;
        }
      }
    } else {
      // direction 1: um = Mhat_1 x, uk = Khat_1 x on every q0 line
      for (int t = threadIdx.x; t < PPB * NC1; t += blockDim.x) {
        const int pp = t / NC1, q0 = t % NC1;
        if (gp0 + pp >= nv) continue;
        T xv[NC1];
#pragma unroll
        for (int j = 0; j < NC1; ++j) xv[j] = xs[pp][q0 + NC1 * j];
#pragma unroll
        for (int r = 1; r <= NP1; ++r) {
          T um = 0, uk = 0;
#pragma unroll
          for (int j = 0; j < NC1; ++j) {
            if (!patch1d_nz<K>(r, j)) continue;
            um += (T)patch1d<K>(m1, r, j) * xv[j];
            uk += (T)patch1d<K>(k1, r, j) * xv[j];
          }
          vm[pp][q0][r - 1] = um;
          vx[pp][q0][r - 1] = uk;
        }
      }
    }
    __syncthreads();
    // direction 0, at the thread's own node: (A x)(node) = Khat_0 vm + Mhat_0 vx
    if (active) {
      const int rw = (pi[1] - 1) + (D == 3 ? NP1 * (pi[2] - 1) : 0);
      T ax = 0;
#pragma unroll
      for (int j = 0; j < NC1; ++j) {
        if (j < pi[0] - K || j > pi[0] + K) continue;
        ax += (T)patch1d_rt<K>(k1, pi[0], j) * vm[p][j][rw];
        ax += (T)patch1d_rt<K>(m1, pi[0], j) * vx[p][j][rw];
      }
      ra[p][i] = bnode - ax;
    }
  }
  __syncthreads();
  // fast diagonalisation: apply S^T along every direction, scale, apply S
  const T* fs = cfs;
  T* src = &ra[0][0];
  T* dst = &rb[0][0];
  for (int stage = 0; stage < 2 * D; ++stage) {
    const int a = stage % D;
    const bool transpose = stage < D;
    if (active) {
      int ia[3];
      int rr = i;
#pragma unroll
      for (int j = 0; j < D; ++j) { ia[j] = rr % NP1; rr /= NP1; }
      int strideA = 1;
      for (int j = 0; j < a; ++j) strideA *= NP1;
      const int baseIdx = i - ia[a] * strideA;
      T s = 0;
#pragma unroll
      for (int q = 0; q < NP1; ++q) {
        const T m = transpose ? fs[q * NP1 + ia[a]] : fs[ia[a] * NP1 + q];
        s += m * src[p * NP + baseIdx + q * strideA];
      }
      if (stage == D - 1) s *= cfd[i];
      dst[p * NP + i] = s;
    }
    __syncthreads();
    T* t = src;
    src = dst;
    dst = t;
  }
  // x at the node is still in the staged closure: no second read of HBM
  if (active) x[node] = xs[p][pi[0] + NC1 * pi[1] + (D == 3 ? NC1 * NC1 * pi[2] : 0)] + src[p * NP + i];
  }
}

template <int D, int K, typename T>
__global__ __launch_bounds__(256) void k_interior_step(KLevel L, const int32_t* __restrict__ verts, int nv,
                                                       T* __restrict__ x, const T* __restrict__ b) {
  interior_step_body<D, K, T>(L, verts, nv, x, b);
}

// argument record of k_interior_step for grouped launches (k_grouped)
template <int D, int K, typename T>
struct InteriorStepArgs {
  KLevel L;
  const int32_t* verts;
  int nv;
  T* x;
  const T* b;
  __device__ void run() const { interior_step_body<D, K, T>(L, verts, nv, x, b); }
};

// Sizes of the cut-patch kernels (one block per patch).
template <int D, int K>
struct CutShape {
  static constexpr int NF = D * 3 * (1 << (D - 1));       // faces touching a 2^d patch
  static constexpr int NT = Pow<K + 1, D - 1>::v;         // nodes of a cell face
  static constexpr int THREADS = Shape<D, K>::NP <= 64 ? 64 : 128;  // one thread per internal node at least
  static constexpr int COPY = 8;                                      // copy-job items per thread of a copy block
  static_assert(Shape<D, K>::NP <= THREADS, "a cut-patch block needs a thread per internal node");
};

// LDS of one cut-patch block.
template <int D, int K, typename T>
struct CutSmem {
  using S = Shape<D, K>;
  using C = CutShape<D, K>;
  double tab[S::T_D1 + K * S::N1 + K - S::T_MHAT];  // mhat | d0 | d1 | gc
  static constexpr int NPAIR = Pow<2 * K, D>::v;  // (node, cell) pairs of a patch, see cut_patch_ax
  // FP64 Q2 in 3-D stages the halo of the ghost faces too (measured faster
  // there; elsewhere the extra staging costs more than the scattered loads)
  static constexpr bool kHalo = sizeof(T) == 8 && D == 3 && K == 2;
  static constexpr int NH = K * Pow<S::NC1, D - 1>::v;  // nodes of one halo slab
  static constexpr int NE = S::NC + (kHalo ? 2 * D * NH : 0);
  T xs[NE];  // x on the patch closure, then the halo slabs (dir, side), see cut_patch_ax
  T Wf[C::NF][K][C::NT];
  T parts[NPAIR];
  int16_t slot[S::NP];  // row of the patch's node at each internal position, -1 if absent
  uint8_t cfl[1 << D], cgh[1 << D];
  int32_t ccut[1 << D];
};

// Patch set-up of the cut-patch kernel: level tables, the 2^d cells around the
// vertex (flags, ghost bits, cut ids) and the vertex coordinates.  Returns the
// lattice node of the thread's internal node (tid < nj), else -1; the slot
// table is filled by cut_patch_ax.
template <int D, int K, typename T>
__device__ int cut_patch_setup(const KLevel& L, const CutGroupDev& G, int gp, CutSmem<D, K, T>& sm, int* V) {
  using S = Shape<D, K>;
  constexpr int N1 = S::N1, NCELL = 1 << D;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int i = tid; i < S::T_D1 + K * N1 + K - S::T_MHAT; i += nth) sm.tab[i] = L.tables[S::T_MHAT + i];
  for (int i = tid; i < S::NP; i += nth) sm.slot[i] = -1;
  const int off = G.off[gp];
  const int nj = G.off[gp + 1] - off;
  const int NV = L.N + 1;
  {
    int vr = G.vertex[gp];
#pragma unroll
    for (int a = 0; a < D; ++a) { V[a] = vr % NV; vr /= NV; }
  }
  if (tid < NCELL) {  // the patch's cells, indexed by the patch (no wait for its vertex)
    const uint16_t fg = G.cell_fg[(int64_t)gp * NCELL + tid];
    sm.cfl[tid] = static_cast<uint8_t>(fg & 0xff);
    sm.cgh[tid] = static_cast<uint8_t>(fg >> 8);
    sm.ccut[tid] = G.cell_cut[(int64_t)gp * NCELL + tid];
  }
  const int node = tid < nj ? G.nodes[off + tid] : -1;  // used after the staging loads are issued
  __syncthreads();  // tables, slot initialisation and cells visible
  return node;
}

// (A x) at the internal node of thread tid (tid < nj; other threads return 0)
// for the patch prepared by cut_patch_setup.  x on the patch closure is staged
// in LDS.  The jumps J_m = d^m-trace(lower) - d^m-trace(upper) of every ghost
// face touching the patch are formed from x in memory (the nodes of both
// cells of the face, which can reach one cell layer beyond the closure) while
// the closure loads are in flight, and contracted with the face mass once per
// face.  The rows are then split into (node, cell) pairs: along each direction
// a node at patch coordinate p in 1..2k-1 lies in cell layer 0 (p <= k) and/or
// 1 (p >= k), which gives 2k (p, layer) choices per direction and (2k)^d pairs,
// enumerated arithmetically (absent nodes and inactive cells give zero).  A
// pair needs its cell row (uncut stiffness or cut-cell matrix) and k (k+1)^{d-1}
// terms per incident ghost face; each node sums its pairs in a fixed order.
// xold receives x at the thread's node.  Called by all threads of the block
// (it synchronises); the LDS buffers are reused on the next call.
template <int D, int K, typename T, int TH>
__device__ T cut_patch_ax(const KLevel& L, int nj, const int* V, int node, int* pi, const T* __restrict__ x,
                          const T* __restrict__ b, CutSmem<D, K, T>& sm, T* xold, T* bval) {
  using S = Shape<D, K>;
  using C = CutShape<D, K>;
  constexpr int N1 = S::N1, NL = S::NL, NC = S::NC, W1 = S::NC1, NF = C::NF, NT = C::NT;
  const int tid = threadIdx.x, nth = blockDim.x;
  const double* mh = sm.tab;
  const double* d0 = sm.tab + (S::T_D0 - S::T_MHAT);
  const double* d1 = sm.tab + (S::T_D1 - S::T_MHAT);
  const double* gc = sm.tab + (S::T_GC - S::T_MHAT);
  if constexpr (CutSmem<D, K, T>::kHalo) {
  // Stage x on the closure and on the halo slabs that ghost faces on the
  // patch boundary need: slab (a, side) holds the k node layers beyond the
  // closure along direction a (cell V-2 for side 0, V+1 for side 1) over the
  // closure's tangential range, node layers fastest.  Coordinates are relative
  // to the closure origin k (V-1).
  constexpr int NH = CutSmem<D, K, T>::NH, NE = CutSmem<D, K, T>::NE;
  uint32_t need = 0;  // bit 2a+side: slab (a, side) is read by a ghost face
#pragma unroll
  for (int o = 0; o < (1 << D); ++o) {
    const uint8_t g = sm.cgh[o];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (((o >> a) & 1) == 0 && (g & (1 << (2 * a)))) need |= 1u << (2 * a);
      if (((o >> a) & 1) == 1 && (g & (1 << (2 * a + 1)))) need |= 1u << (2 * a + 1);
    }
  }
  constexpr int NIT = (NE + TH - 1) / TH;
  T v[NIT];
#pragma unroll
  for (int u = 0; u < NIT; ++u) {
    const int e = tid + TH * u;
    v[u] = 0;
    int rr[3];
    bool ld = e < NE;
    if (e < NC) {
      int r = e;
#pragma unroll
      for (int a = 0; a < D; ++a) { rr[a] = r % W1; r /= W1; }
    } else if (ld) {
      const int h = e - NC, slab = h / NH, dir = slab >> 1, side = slab & 1;
      int r = h % NH;
      const int layer = r % K;
      r /= K;
      ld = ((need >> slab) & 1) && !L.ghost_local;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        if (a == dir) {
          rr[a] = side ? 2 * K + 1 + layer : layer - K;
        } else {
          rr[a] = r % W1;
          r /= W1;
        }
      }
    }
    if (ld) {
      int I[3];
      bool in = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        I[a] = K * (V[a] - 1) + rr[a];
        in = in && I[a] >= 0 && I[a] < L.nn;
      }
      if (in) v[u] = x[lat(D, L.nn, I)];
    }
  }
  // the thread's node (its load was issued in the set-up): patch coordinates
  // 1 .. 2k-1, row in the slot table, and b, whose load overlaps the staging
  if (tid < nj) {
    int r = node, pos = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pi[a] = r % L.nn - K * (V[a] - 1);
      r /= L.nn;
    }
#pragma unroll
    for (int a = D - 1; a >= 0; --a) pos = pos * S::NP1 + (pi[a] - 1);
    sm.slot[pos] = static_cast<int16_t>(tid);
    *bval = b[node];
  }
#pragma unroll
  for (int u = 0; u < NIT; ++u) {
    const int e = tid + TH * u;
    if (e < NE) sm.xs[e] = v[u];
  }
  __syncthreads();
  // mass-contracted jumps W_m(i_t) of every ghost face touching the patch:
  // face (dir, plane 0..2, tangential cell t), plane p between cell layers p-1, p
  for (int task = tid; task < NF * K; task += nth) {
    const int m = task % K;
    const int f = task / K;
    const int dir = f / (3 << (D - 1));
    const int plane = (f >> (D - 1)) % 3;
    const int t = f & ((1 << (D - 1)) - 1);
    int o = 0, tb = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (a == dir) continue;
      o |= ((t >> tb) & 1) << a;
      ++tb;
    }
    bool ghost;
    if (plane == 0) ghost = sm.cgh[o] & (1 << (2 * dir));               // lower face of layer 0
    else if (plane == 1) ghost = sm.cgh[o] & (1 << (2 * dir + 1));      // between layers 0 and 1
    else ghost = sm.cgh[o | (1 << dir)] & (1 << (2 * dir + 1));         // upper face of layer 1
    if (!ghost) continue;
    // closure strides of the normal (sd) and tangential (s0, s1) directions
    // and the tangential cell offsets (K t0, K t1) of the face
    int sd = 1, s0 = 0, s1 = 0, k0 = 0, k1 = 0, tb2 = 0, st = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (a == dir) {
        sd = st;
      } else if (tb2 == 0) {
        s0 = st;
        k0 = K * ((t >> tb2) & 1);
        ++tb2;
      } else {
        s1 = st;
        k1 = K * ((t >> tb2) & 1);
        ++tb2;
      }
      st *= W1;
    }
    const int hbase = NC + 2 * dir * NH;
    T dl[N1], du[N1];
#pragma unroll
    for (int bd = 0; bd <= K; ++bd) {
      dl[bd] = (T)d1[m * N1 + bd];
      du[bd] = (T)d0[m * N1 + bd];
    }
    // LDS index of the node with normal coordinate rd (first node of the lower
    // cell at K (plane - 1)) and tangential coordinates (r0, r1)
    auto idx = [&](int rd, int r0, int r1) {
      if (rd >= 0 && rd <= 2 * K) return r0 * s0 + r1 * s1 + rd * sd;
      const int side = rd > 2 * K;
      return hbase + side * NH + (r0 + W1 * r1) * K + (side ? rd - 2 * K - 1 : rd + K);
    };
    T J[NT];
#pragma unroll
    for (int bt = 0; bt < NT; ++bt) {
      const int r0 = k0 + bt % N1, r1 = D == 3 ? k1 + bt / N1 : 0;
      T acc0 = 0, acc1 = 0;
#pragma unroll
      for (int bd = 0; bd <= K; ++bd) {
        acc0 += dl[bd] * sm.xs[idx(K * (plane - 1) + bd, r0, r1)];
        acc1 += du[bd] * sm.xs[idx(K * plane + bd, r0, r1)];
      }
      J[bt] = acc0 - acc1;
    }
    T mm[N1 * N1];
#pragma unroll
    for (int i = 0; i < N1 * N1; ++i) mm[i] = (T)mh[i];
    if (D == 2) {
#pragma unroll
      for (int it = 0; it < N1; ++it) {
        T acc = 0;
#pragma unroll
        for (int bt = 0; bt < N1; ++bt) acc += mm[it * N1 + bt] * J[bt];
        sm.Wf[f][m][it] = acc;
      }
    } else {
      // (Mhat x Mhat) J by two 1-D contractions
      T H[NT];
#pragma unroll
      for (int b1 = 0; b1 < N1; ++b1)
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) {
          T acc = 0;
#pragma unroll
          for (int b0 = 0; b0 < N1; ++b0) acc += mm[i0 * N1 + b0] * J[b0 + N1 * b1];
          H[i0 + N1 * b1] = acc;
        }
#pragma unroll
      for (int i1 = 0; i1 < N1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) {
          T acc = 0;
#pragma unroll
          for (int b1 = 0; b1 < N1; ++b1) acc += mm[i1 * N1 + b1] * H[i0 + N1 * b1];
          sm.Wf[f][m][i0 + N1 * i1] = acc;
        }
    }
  }
  } else {
  const int64_t nn = L.nn;
  // closure loads first (stored to LDS after the face jumps; blockDim == THREADS)
  constexpr int NIT = (NC + TH - 1) / TH;
  T v[NIT];
#pragma unroll
  for (int u = 0; u < NIT; ++u) {
    const int e = tid + TH * u;
    v[u] = 0;
    if (e < NC) {
      int I[3], r = e;
      bool in = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        I[a] = K * (V[a] - 1) + r % W1;
        r /= W1;
        in = in && I[a] >= 0 && I[a] < L.nn;
      }
      if (in) v[u] = x[lat(D, L.nn, I)];
    }
  }
  // the thread's node (its load was issued in the set-up): patch coordinates
  // 1 .. 2k-1, row in the slot table, and b, whose load overlaps the staging
  if (tid < nj) {
    int r = node, pos = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pi[a] = r % L.nn - K * (V[a] - 1);
      r /= L.nn;
    }
#pragma unroll
    for (int a = D - 1; a >= 0; --a) pos = pos * S::NP1 + (pi[a] - 1);
    sm.slot[pos] = static_cast<int16_t>(tid);
    *bval = b[node];
  }
  // mass-contracted jumps W_m(i_t) of every ghost face touching the patch:
  // face (dir, plane 0..2, tangential cell t), plane p between cell layers p-1, p
  for (int task = tid; task < NF * K; task += nth) {
    const int m = task % K;
    const int f = task / K;
    const int dir = f / (3 << (D - 1));
    const int plane = (f >> (D - 1)) % 3;
    const int t = f & ((1 << (D - 1)) - 1);
    int o = 0, tb = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (a == dir) continue;
      o |= ((t >> tb) & 1) << a;
      ++tb;
    }
    bool ghost;
    if (plane == 0) ghost = sm.cgh[o] & (1 << (2 * dir));               // lower face of layer 0
    else if (plane == 1) ghost = sm.cgh[o] & (1 << (2 * dir + 1));      // between layers 0 and 1
    else ghost = sm.cgh[o | (1 << dir)] & (1 << (2 * dir + 1));         // upper face of layer 1
    if (!ghost) continue;
    // first node of the lower cell of the face, lattice strides of the
    // tangential directions and of the normal one (a ghost face has both of
    // its cells in the background box, so every node read is in the lattice)
    int I[3], tb2 = 0;
    int64_t st0 = 0, st1 = 0, sn = 1, sa = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (a == dir) {
        I[a] = K * (V[a] - 2 + plane);
        sn = sa;
      } else {
        I[a] = K * (V[a] - 1 + ((t >> tb2) & 1));
        if (tb2 == 0) st0 = sa; else st1 = sa;
        ++tb2;
      }
      sa *= nn;
    }
    const int64_t base = lat(D, L.nn, I);
    // patch-local residual: the lower cell of a plane-0 face and the upper
    // cell of a plane-2 face lie outside the patch; their nodes beyond the
    // closure (normal layers other than the shared face) get weight zero (the
    // loads stay unconditional)
    const bool lo_out = L.ghost_local && plane == 0, hi_out = L.ghost_local && plane == 2;
    T dl[N1], du[N1];
#pragma unroll
    for (int bd = 0; bd <= K; ++bd) {
      dl[bd] = (lo_out && bd < K) ? (T)0 : (T)d1[m * N1 + bd];
      du[bd] = (hi_out && bd > 0) ? (T)0 : (T)d0[m * N1 + bd];
    }
    T J[NT];
#pragma unroll
    for (int bt = 0; bt < NT; ++bt) {
      const int64_t el = base + (bt % N1) * st0 + (D == 3 ? (bt / N1) * st1 : 0);
      T acc0 = 0, acc1 = 0;
#pragma unroll
      for (int bd = 0; bd <= K; ++bd) {
        acc0 += dl[bd] * x[el + bd * sn];
        acc1 += du[bd] * x[el + (bd + K) * sn];
      }
      J[bt] = acc0 - acc1;
    }
    T mm[N1 * N1];
#pragma unroll
    for (int i = 0; i < N1 * N1; ++i) mm[i] = (T)mh[i];
    if (D == 2) {
#pragma unroll
      for (int it = 0; it < N1; ++it) {
        T acc = 0;
#pragma unroll
        for (int bt = 0; bt < N1; ++bt) acc += mm[it * N1 + bt] * J[bt];
        sm.Wf[f][m][it] = acc;
      }
    } else {
      // (Mhat x Mhat) J by two 1-D contractions
      T H[NT];
#pragma unroll
      for (int b1 = 0; b1 < N1; ++b1)
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) {
          T acc = 0;
#pragma unroll
          for (int b0 = 0; b0 < N1; ++b0) acc += mm[i0 * N1 + b0] * J[b0 + N1 * b1];
          H[i0 + N1 * b1] = acc;
        }
#pragma unroll
      for (int i1 = 0; i1 < N1; ++i1)
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) {
          T acc = 0;
#pragma unroll
          for (int b1 = 0; b1 < N1; ++b1) acc += mm[i1 * N1 + b1] * H[i0 + N1 * b1];
          sm.Wf[f][m][i0 + N1 * i1] = acc;
        }
    }
  }
#pragma unroll
  for (int u = 0; u < NIT; ++u) {
    const int e = tid + TH * u;
    if (e < NC) sm.xs[e] = v[u];
  }
  }
  __syncthreads();
  // (node, cell) pairs
  constexpr int NPAIR = CutSmem<D, K, T>::NPAIR;
  for (int t = tid; t < NPAIR; t += nth) {
    int p[3], o = 0, pos = 0;
    {
      int r = t;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int j = r % (2 * K);
        r /= 2 * K;
        p[a] = j < K ? j + 1 : j;
        o |= (j >= K ? 1 : 0) << a;
      }
#pragma unroll
      for (int a = D - 1; a >= 0; --a) pos = pos * S::NP1 + (p[a] - 1);
    }
    T part = 0;
    const uint8_t f = sm.cfl[o];
    if (sm.slot[pos] >= 0 && (f & 1)) {
      int il[3];
#pragma unroll
      for (int a = 0; a < D; ++a) il[a] = p[a] - K * ((o >> a) & 1);
      int iloc = il[0] + N1 * il[1];
      if (D == 3) iloc += N1 * N1 * il[2];
      int xb = K * (o & 1) + W1 * K * ((o >> 1) & 1);  // closure index of the cell's first node
      if (D == 3) xb += W1 * W1 * K * ((o >> 2) & 1);
      // dot product of the cell row with x, one partial sum per x-row of the cell
      constexpr int NRW = N1 * (D == 3 ? N1 : 1);
      T acc[NRW];
#pragma unroll
      for (int a = 0; a < NRW; ++a) acc[a] = 0;
      if (f & 2) {
        const T* row = L.cut_mats_t<T>() + ((int64_t)sm.ccut[o] * NL + iloc) * NL;
#pragma unroll
        for (int bq = 0; bq < NL; ++bq) {
          const int b0 = bq % N1, b12 = bq / N1;
          const int xi = xb + b0 + W1 * (b12 % N1) + (D == 3 ? W1 * W1 * (b12 / N1) : 0);
          acc[b12] += row[bq] * sm.xs[xi];
        }
      } else {
        const T* row = L.kcell_t<T>() + S::T_KCELL + iloc * NL;
#pragma unroll
        for (int bq = 0; bq < NL; ++bq) {
          const int b0 = bq % N1, b12 = bq / N1;
          const int xi = xb + b0 + W1 * (b12 % N1) + (D == 3 ? W1 * W1 * (b12 / N1) : 0);
          acc[b12] += row[bq] * sm.xs[xi];
        }
      }
#pragma unroll
      for (int a = 0; a < NRW; ++a) part += acc[a];
      const uint8_t g = sm.cgh[o];
      if (g) {
#pragma unroll
        for (int dir = 0; dir < D; ++dir)
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            if (!(g & (1 << (2 * dir + side)))) continue;
            const int plane = ((o >> dir) & 1) + side;
            int tt = 0, tb = 0, it = 0, st = 1;
#pragma unroll
            for (int a = 0; a < D; ++a) {
              if (a == dir) continue;
              tt |= ((o >> a) & 1) << tb;
              ++tb;
              it += il[a] * st;
              st *= N1;
            }
            const int fi = (dir * 3 + plane) * (1 << (D - 1)) + tt;
#pragma unroll
            for (int m = 0; m < K; ++m) {
              const double sg = gc[m] * (side == 1 ? d1[m * N1 + il[dir]] : -d0[m * N1 + il[dir]]);
              part += (T)sg * sm.Wf[fi][m][it];
            }
          }
      }
    }
    sm.parts[t] = part;
  }
  __syncthreads();
  T ax = 0;
  if (tid < nj) {
    // x at the node itself (closure index = patch coordinates)
    *xold = sm.xs[pi[0] + W1 * pi[1] + (D == 3 ? W1 * W1 * pi[2] : 0)];
    // the node's pairs: per direction index j = p - 1 (layer 0, p <= k) and
    // j = p (layer 1, p >= k), in increasing pair index
    int jlo[3], jn[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      jlo[a] = pi[a] <= K ? pi[a] - 1 : pi[a];
      jn[a] = pi[a] == K ? 2 : 1;
    }
    const int ncomb = jn[0] * jn[1] * (D == 3 ? jn[2] : 1);
    for (int comb = 0; comb < ncomb; ++comb) {
      int t = 0, r = comb, st = 1;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int sel = r % jn[a];
        r /= jn[a];
        t += (jlo[a] + sel) * st;
        st *= 2 * K;
      }
      ax += sm.parts[t];
    }
  }
  __syncthreads();  // the buffers may be restaged by the next call
  return ax;
}

// Cut patches, phase 1: residual on the internal nodes and dense local solve
// d_j = A_j^{-1} r_j (GEMV with the symmetric inverse), one block per patch
// and one column per blockIdx.y (columns are n_nodes apart in x, b and xb and
// n_nodes of the colour apart in dbuf).  With xb == nullptr d_j goes to dbuf;
// otherwise xb = x + d_j on the patch's internal DoFs (same-coloured patches
// share none), and the first cj.nblk blocks copy the nodes of the copy job
// from x to xb instead of solving a patch.
template <int D, int K, typename T, int TH>
__global__ __launch_bounds__(TH) void k_cut_solve(KLevel L, CutGroupDev G,
                                                                        const T* __restrict__ x,
                                                                        const T* __restrict__ b,
                                                                        T* __restrict__ dbuf, T* __restrict__ xb,
                                                                        CopyJob cj) {
  using S = Shape<D, K>;
  using C = CutShape<D, K>;
  __shared__ CutSmem<D, K, T> sm;
  constexpr int RSN = (S::NP + 31) / 32 * 32;  // residual rows, padded with zeros to whole GEMV batches
  __shared__ T rs[RSN];
  const int tid = threadIdx.x;
  x += blockIdx.y * L.n_nodes;
  b += blockIdx.y * L.n_nodes;
  dbuf += blockIdx.y * G.n_nodes;
  if (xb) xb += blockIdx.y * L.n_nodes;
  if ((int)blockIdx.x < cj.nblk) {
    // copy block: C::COPY items per thread, index loads first, then the values
    int32_t nd[C::COPY];
#pragma unroll
    for (int u = 0; u < C::COPY; ++u) {
      const int64_t i = ((int64_t)blockIdx.x * C::COPY + u) * TH + tid;
      nd[u] = (i < cj.n && !(cj.skip[i] & cj.mask)) ? cj.nodes[i] : -1;
    }
    T v[C::COPY];
#pragma unroll
    for (int u = 0; u < C::COPY; ++u) v[u] = nd[u] >= 0 ? x[nd[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < C::COPY; ++u)
      if (nd[u] >= 0) xb[nd[u]] = v[u];
    return;
  }
  const int gp = xcd_block(blockIdx.x - cj.nblk, gridDim.x - cj.nblk);
  int V[3] = {0, 0, 0}, pi[3] = {0, 0, 0};
  const int node = cut_patch_setup<D, K, T>(L, G, gp, sm, V);
  const int off = G.off[gp];
  const int nj = G.off[gp + 1] - off;
  T xold = 0, bval = 0;
  const T ax = cut_patch_ax<D, K, T, TH>(L, nj, V, node, pi, x, b, sm, &xold, &bval);
  if (tid < nj) rs[tid] = bval - ax;
  for (int e = nj + tid; e < RSN; e += TH) rs[e] = 0;
  __syncthreads();
  // d = A_j^{-1} r: thread i takes row i (= column i, the inverse is symmetric)
  // (blockDim >= NP >= nj).  Small patches issue all loads of the row at once,
  // larger ones in batches; loads past the last row re-read it (their
  // residual entries are zero), so every load of a batch is issued unconditionally.
  if (tid >= nj) return;
  const T* inv = G.inv_t<T>() + G.inv_off[gp];
  T dv;
  if constexpr (S::NP <= 32) {
    T v[S::NP];
#pragma unroll
    for (int j = 0; j < S::NP; ++j) v[j] = inv[(int64_t)(j < nj ? j : nj - 1) * nj + tid];
    T acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < S::NP; ++j) acc[j % 4] += v[j] * rs[j];
    dv = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  } else {
    // batches of 32 (FP32) or 16 (FP64) independent loads
    constexpr int NB = sizeof(T) == 4 ? 32 : 16;
    const int i = tid;
    T acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0;
    for (int j = 0; j < nj; j += NB) {
      T v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) v[u] = inv[(int64_t)(j + u < nj ? j + u : nj - 1) * nj + i];
#pragma unroll
      for (int u = 0; u < NB; ++u) acc[u % 8] += v[u] * rs[j + u];
    }
    dv = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  if (xb)
    xb[node] = xold + dv;
  else
    dbuf[off + tid] = dv;
}

// Residual rows of one cut patch for NCOL columns at once.  The patch closure
// of every column is staged node-major in LDS (the columns of a node
// adjacent).  The work is split into (node, cell) pairs: along each direction
// an internal node at patch coordinate p in 1..2k-1 lies in cell layer 0
// (p <= k) and/or 1 (p >= k), which gives 2k (p, layer) choices per direction
// and (2k)^d pairs per patch, enumerated arithmetically (pairs of absent nodes
// or inactive cells contribute zero).  A pair applies its cell row (cut-cell
// matrix or uncut stiffness, read once for all columns) and the ghost-face
// terms of that cell (from the level's face buffer W, written by k_face_w for
// the current x just before) to all columns, into parts[pair][column]; each
// node then sums its 1..2^d pairs in a fixed order.  Every column follows the
// same arithmetic in the same order, so its result does not depend on the
// other columns.  Returns the residual rows in the LDS of the staged closure
// (free once the pairs are formed): rs[i][c] = b_c - (A x_c) at node i for
// i < nj and c < ncol, zero elsewhere in the first nrows rows (nrows <= the
// closure's node count).  All threads of the block call it (it synchronises).
template <int D, int K, typename T, int NCOL>
struct PairSmem {
  using S = Shape<D, K>;
  static constexpr int NPAIR = Pow<2 * K, D>::v;
  double tab[S::T_GC + K - S::T_D0];  // d0 | d1 | gc
  T xs[S::NC][NCOL];
  T parts[NPAIR][NCOL];
  int16_t slot[S::NP];  // row of the patch's node at each internal position, -1 if absent
  uint8_t cfl[1 << D], cgh[1 << D];
  int32_t ccut[1 << D], cgid[1 << D];
};

template <int D, int K, typename T, int NCOL>
__device__ void cut_residual_cols(const KLevel& L, const CutGroupDev& G, int gp, const T* __restrict__ x,
                                  const T* __restrict__ b, const T* __restrict__ W, int ncol,
                                  PairSmem<D, K, T, NCOL>& sm, int nrows, int& off, int& nj) {
  using S = Shape<D, K>;
  constexpr int N1 = S::N1, NL = S::NL, NC = S::NC, NC1 = S::NC1, NP1 = S::NP1, NCELL = 1 << D;
  constexpr int NT = Pow<N1, D - 1>::v;
  constexpr int NTAB = S::T_GC + K - S::T_D0;
  constexpr int NPAIR = PairSmem<D, K, T, NCOL>::NPAIR;
  constexpr int TH = CutShape<D, K>::THREADS;
  const int tid = threadIdx.x;
  for (int i = tid; i < NTAB; i += TH) sm.tab[i] = L.tables[S::T_D0 + i];
  for (int i = tid; i < S::NP; i += TH) sm.slot[i] = -1;
  const double* d0 = sm.tab;
  const double* d1 = sm.tab + K * N1;
  const double* gc = sm.tab + 2 * K * N1;
  off = G.off[gp];
  nj = G.off[gp + 1] - off;
  const int NV = L.N + 1;
  int V[3] = {0, 0, 0};
  {
    int vr = G.vertex[gp];
#pragma unroll
    for (int a = 0; a < D; ++a) { V[a] = vr % NV; vr /= NV; }
  }
  const int64_t nn = L.nn, nn2 = nn * nn;
  const int64_t cbase = K * (V[0] - 1) + nn * (K * (V[1] - 1)) + (D == 3 ? nn2 * (K * (V[2] - 1)) : 0);
  if (tid < NCELL) {
    int c[3];
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      c[a] = V[a] - 1 + ((tid >> a) & 1);
      in = in && c[a] >= 0 && c[a] < L.N;
    }
    uint8_t f = 0, g = 0;
    int32_t cid = -1, gid = -1;
    if (in) {
      const int64_t cl = cell_lin(D, L.N, c);
      f = L.flags[cl];
      g = L.ghost[cl];
      cid = L.cut_id[cl];
      gid = L.cell_gid[cl];
    }
    sm.cfl[tid] = f;
    sm.cgh[tid] = g;
    sm.ccut[tid] = cid;
    sm.cgid[tid] = gid;
  }
  // node, patch position and b of the thread's row, fetched before the staging
  int pi[3] = {0, 0, 0};
  T bv[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) bv[c] = 0;
  if (tid < nj) {
    const int node = G.nodes[off + tid];
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
      if (c < ncol) bv[c] = b[c * L.n_nodes + node];
    int r = node;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pi[a] = r % L.nn - K * (V[a] - 1);
      r /= L.nn;
    }
  }
  // stage the closure of every column (nodes outside the lattice are zero);
  // all loads of a thread are issued before its LDS stores
  {
    constexpr int NST = NC * NCOL;
    constexpr int NIT = (NST + TH - 1) / TH;
    T v[NIT];
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = tid + TH * u;
      v[u] = 0;
      const int q = e / NCOL, c = e % NCOL;
      if (e < NST && c < ncol) {
        const int q0 = q % NC1, q1 = (q / NC1) % NC1, q2 = q / (NC1 * NC1);
        const int I0 = K * (V[0] - 1) + q0, I1 = K * (V[1] - 1) + q1, I2 = D == 3 ? K * (V[2] - 1) + q2 : 0;
        const bool in = I0 >= 0 && I0 < nn && I1 >= 0 && I1 < nn && (D == 2 || (I2 >= 0 && I2 < nn));
        if (in) v[u] = x[c * L.n_nodes + cbase + q0 + nn * q1 + (D == 3 ? nn2 * q2 : 0)];
      }
    }
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = tid + TH * u;
      if (e < NST) sm.xs[e / NCOL][e % NCOL] = v[u];
    }
  }
  if (tid < nj) {
    int pos = 0;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) pos = pos * NP1 + (pi[a] - 1);
    sm.slot[pos] = static_cast<int16_t>(tid);
  }
  __syncthreads();
  const int64_t wcol = L.n_faces * K * NT;
  for (int t = tid; t < NPAIR; t += TH) {
    int p[3], o = 0, pos = 0;
    {
      int r = t;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int j = r % (2 * K);
        r /= 2 * K;
        const int layer = j >= K ? 1 : 0;
        p[a] = j < K ? j + 1 : j;
        o |= layer << a;
      }
#pragma unroll
      for (int a = D - 1; a >= 0; --a) pos = pos * NP1 + (p[a] - 1);
    }
    T acc[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) acc[c] = 0;
    const uint8_t f = sm.cfl[o];
    if (sm.slot[pos] >= 0 && (f & 1)) {
      int il[3];
#pragma unroll
      for (int a = 0; a < D; ++a) il[a] = p[a] - K * ((o >> a) & 1);
      int iloc = il[0] + N1 * il[1];
      if (D == 3) iloc += N1 * N1 * il[2];
      int qb = K * (o & 1) + NC1 * K * ((o >> 1) & 1);  // closure index of the cell's first node
      if (D == 3) qb += NC1 * NC1 * K * ((o >> 2) & 1);
      if (f & 2) {
        const T* row = L.cut_mats_t<T>() + ((int64_t)sm.ccut[o] * NL + iloc) * NL;
#pragma unroll 8
        for (int bq = 0; bq < NL; ++bq) {
          const int b0 = bq % N1, b12 = bq / N1;
          const int q = qb + b0 + NC1 * (b12 % N1) + (D == 3 ? NC1 * NC1 * (b12 / N1) : 0);
          const T m = row[bq];
#pragma unroll
          for (int c = 0; c < NCOL; ++c) acc[c] += m * sm.xs[q][c];
        }
      } else {
        const T* row = L.kcell_t<T>() + S::T_KCELL + iloc * NL;
#pragma unroll 8
        for (int bq = 0; bq < NL; ++bq) {
          const int b0 = bq % N1, b12 = bq / N1;
          const int q = qb + b0 + NC1 * (b12 % N1) + (D == 3 ? NC1 * NC1 * (b12 / N1) : 0);
          const T m = row[bq];
#pragma unroll
          for (int c = 0; c < NCOL; ++c) acc[c] += m * sm.xs[q][c];
        }
      }
      const uint8_t g = sm.cgh[o];
      if (g) {
        const int gid = sm.cgid[o];
#pragma unroll
        for (int dir = 0; dir < D; ++dir)
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            if (!(g & (1 << (2 * dir + side)))) continue;
            const int fid = L.cell_faces[(int64_t)gid * 2 * D + 2 * dir + side];
            int it = 0, st = 1;
#pragma unroll
            for (int a = 0; a < D; ++a) {
              if (a == dir) continue;
              it += il[a] * st;
              st *= N1;
            }
            const T* w = W + (int64_t)fid * K * NT + it;
#pragma unroll
            for (int m = 0; m < K; ++m) {
              const T sg = (T)(gc[m] * (side == 1 ? d1[m * N1 + il[dir]] : -d0[m * N1 + il[dir]]));
#pragma unroll
              for (int c = 0; c < NCOL; ++c)
                if (c < ncol) acc[c] += sg * w[c * wcol + m * NT];
            }
          }
      }
    }
#pragma unroll
    for (int c = 0; c < NCOL; ++c) sm.parts[t][c] = acc[c];
  }
  __syncthreads();
  if (tid < nj) {
    // the node's pairs: per direction index j = p - 1 (layer 0, p <= k) and
    // j = p (layer 1, p >= k), in increasing pair index
    int jlo[3], jn[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      jlo[a] = pi[a] <= K ? pi[a] - 1 : pi[a];
      jn[a] = pi[a] == K ? 2 : 1;
    }
    T acc[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) acc[c] = 0;
    const int ncomb = jn[0] * jn[1] * (D == 3 ? jn[2] : 1);
    for (int comb = 0; comb < ncomb; ++comb) {
      int t = 0, r = comb, st = 1;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int sel = r % jn[a];
        r /= jn[a];
        t += (jlo[a] + sel) * st;
        st *= 2 * K;
      }
#pragma unroll
      for (int c = 0; c < NCOL; ++c) acc[c] += sm.parts[t][c];
    }
    T(*rs)[NCOL] = sm.xs;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) rs[tid][c] = c < ncol ? bv[c] - acc[c] : (T)0;
  }
  for (int e = nj * NCOL + tid; e < nrows * NCOL; e += TH) (&sm.xs[0][0])[e] = 0;
  __syncthreads();
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Cut patches, phase 1 for up to kMaxCols columns in FP32, local solves on the
// matrix cores.  Residuals of all columns by cut_residual_cols, then
// D = A_j^{-1} R with v_mfma_f32_16x16x4f32, which multiplies a 16x4 tile of
// the inverse (lane l holds row l%16, column l/16) by a 4x16 slice of R (lane
// l holds row l/16, column l%16; columns >= kMaxCols are zero) into 16x16
// accumulators (lane l holds rows 4(l/16)..4(l/16)+3 of column l%16).  The
// inverse is stored tile by tile in exactly that lane order
// (CutGroupDev::inv_tiles), so a tile is one coalesced 256-byte wave load, and
// it is read once for all columns.  Row blocks of 16 are spread over the
// block's wavefronts.
template <int D, int K>
__device__ __forceinline__ void cut_solve_mfma_body(KLevel L, CutGroupDev G, const float* __restrict__ x,
                                                    const float* __restrict__ b, const float* __restrict__ W,
                                                    float* __restrict__ dbuf, int ncol) {
  using S = Shape<D, K>;
  constexpr int NPK = (S::NP + 3) / 4 * 4;
  __shared__ PairSmem<D, K, float, kMaxCols> sm;
  static_assert(NPK <= S::NC, "the residual rows fit in the staged closure");
  const int tid = threadIdx.x, nth = blockDim.x;
  const int gp = xcd_block(blockIdx.x, gridDim.x);
  if (gp >= G.n_patch) return;  // grouped launches: a block beyond this problem's patches
  int off, nj;
  cut_residual_cols<D, K, float, kMaxCols>(L, G, gp, x, b, W, ncol, sm, NPK, off, nj);
  // residual columns; rows >= nj and columns >= ncol are zero
  const float(*rs)[kMaxCols] = sm.xs;
  const int lane = tid % 64, wave = tid / 64, nwave = nth / 64;
  const int nrb = (nj + 15) / 16, nkb = (nj + 3) / 4;
  const int kr = lane / 16, jc = lane % 16;
  const float* tiles = G.inv_tiles + G.tile_off[gp];
  // all tiles of a row block are loaded at once (NKB <= 32 registers), then
  // the MFMA chain runs on them
  constexpr int NKB = NPK / 4;
  for (int rb = wave; rb < nrb; rb += nwave) {  // wave-uniform: every lane takes part in the MFMA
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* t = tiles + (int64_t)rb * nkb * 64 + lane;
    float a[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) a[kb] = kb < nkb ? t[kb * 64] : 0.f;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      if (kb < nkb) {
        const float bb = jc < kMaxCols ? rs[kb * 4 + kr][jc] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kb], bb, acc, 0, 0, 0);
      }
    }
    if (jc < ncol) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = rb * 16 + 4 * kr + v;
        if (i < nj) dbuf[jc * G.n_nodes + off + i] = acc[v];
      }
    }
  }
}

template <int D, int K>
__global__ __launch_bounds__((CutShape<D, K>::THREADS)) void k_cut_solve_mfma(KLevel L, CutGroupDev G,
                                                                              const float* __restrict__ x,
                                                                              const float* __restrict__ b,
                                                                              const float* __restrict__ W,
                                                                              float* __restrict__ dbuf, int ncol) {
  cut_solve_mfma_body<D, K>(L, G, x, b, W, dbuf, ncol);
}

// argument record of k_cut_solve_mfma for grouped launches (k_grouped)
template <int D, int K>
struct CutSolveMfmaArgs {
  KLevel L;
  CutGroupDev G;
  const float* x;
  const float* b;
  const float* W;
  float* dbuf;
  int ncol;
  __device__ void run() const { cut_solve_mfma_body<D, K>(L, G, x, b, W, dbuf, ncol); }
};

// Cut patches, phase 1 for up to kMaxCols columns in FP64: residuals of all
// columns by cut_residual_cols (every cell row read once for all columns),
// then d = A_j^{-1} r for all columns with the inverse read once: thread i
// takes row i (= column i, the inverse is symmetric) and multiplies each entry
// into every column's accumulator.  Column c's arithmetic (residual, then the
// row sum in increasing j) does not depend on the other columns.
template <int D, int K>
__device__ __forceinline__ void cut_solve_cols_body(KLevel L, CutGroupDev G, const double* __restrict__ x,
                                                    const double* __restrict__ b, const double* __restrict__ W,
                                                    double* __restrict__ dbuf, int ncol) {
  using S = Shape<D, K>;
  constexpr int NB = 8;                        // independent inverse loads in flight per thread
  constexpr int NPB = (S::NP + NB - 1) / NB * NB;
  __shared__ PairSmem<D, K, double, kMaxCols> sm;
  static_assert(NPB <= S::NC, "the residual rows fit in the staged closure");
  const int tid = threadIdx.x, nth = blockDim.x;
  const int gp = xcd_block(blockIdx.x, gridDim.x);
  if (gp >= G.n_patch) return;  // grouped launches: a block beyond this problem's patches
  int off, nj;
  cut_residual_cols<D, K, double, kMaxCols>(L, G, gp, x, b, W, ncol, sm, NPB, off, nj);
  const double(*rs)[kMaxCols] = sm.xs;  // rows >= nj and columns >= ncol are zero
  const double* inv = G.inv_t<double>() + G.inv_off[gp];
  for (int i = tid; i < nj; i += nth) {
    double acc[kMaxCols];
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c) acc[c] = 0.0;
    for (int j = 0; j < nj; j += NB) {
      double v[NB];
      // loads past the last row re-read it; their residual rows are zero
#pragma unroll
      for (int u = 0; u < NB; ++u) v[u] = inv[(int64_t)(j + u < nj ? j + u : nj - 1) * nj + i];
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int c = 0; c < kMaxCols; ++c) acc[c] += v[u] * rs[j + u][c];
    }
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c)
      if (c < ncol) dbuf[c * G.n_nodes + off + i] = acc[c];
  }
}

template <int D, int K>
__global__ __launch_bounds__((CutShape<D, K>::THREADS)) void k_cut_solve_cols(KLevel L, CutGroupDev G,
                                                                              const double* __restrict__ x,
                                                                              const double* __restrict__ b,
                                                                              const double* __restrict__ W,
                                                                              double* __restrict__ dbuf, int ncol) {
  cut_solve_cols_body<D, K>(L, G, x, b, W, dbuf, ncol);
}

// argument record of k_cut_solve_cols for grouped launches (k_grouped)
template <int D, int K>
struct CutSolveColsArgs {
  KLevel L;
  CutGroupDev G;
  const double* x;
  const double* b;
  const double* W;
  double* dbuf;
  int ncol;
  __device__ void run() const { cut_solve_cols_body<D, K>(L, G, x, b, W, dbuf, ncol); }
};

// dst = src on a node list (the cut region before a run of two-buffer cut steps).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_nodes(const int32_t* __restrict__ nodes, int64_t n,
                                                    const T* __restrict__ src, T* __restrict__ dst, int64_t ld) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) {
    const int64_t o = blockIdx.y * ld + nodes[e];
    dst[o] = src[o];
  }
}

// Cut patches, phase 2: x[I_j] += d_j for all patches of the colour.
template <typename T>
__device__ __forceinline__ void cut_update_body(const int32_t* __restrict__ nodes, int64_t n,
                                                const T* __restrict__ dbuf, T* __restrict__ x, int64_t ldx) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) x[blockIdx.y * ldx + nodes[e]] += dbuf[blockIdx.y * n + e];
}

template <typename T>
__global__ __launch_bounds__(256) void k_cut_update(const int32_t* __restrict__ nodes, int64_t n,
                                                    const T* __restrict__ dbuf, T* __restrict__ x, int64_t ldx) {
  cut_update_body<T>(nodes, n, dbuf, x, ldx);
}

// argument record of k_cut_update for grouped launches (k_grouped)
template <typename T>
struct CutUpdateArgs {
  const int32_t* nodes;
  int64_t n;
  const T* dbuf;
  T* x;
  int64_t ldx;
  __device__ void run() const { cut_update_body<T>(nodes, n, dbuf, x, ldx); }
};

// x_f[I] += sum_J P(I, J) x_c[J] for every active fine node (embedding).
template <int D, int K, typename T>
__device__ __forceinline__ void prolong_add_body(KLevel Lc, KLevel Lf, const T* __restrict__ xc, T* __restrict__ xf) {
  using S = Shape<D, K>;
  constexpr int N1 = S::N1;
  __shared__ double p1d[S::NC1 * N1];
  for (int t = threadIdx.x; t < S::NC1 * N1; t += blockDim.x) p1d[t] = Lf.tables[S::T_P1D + t];
  __syncthreads();
  xc += blockIdx.y * Lc.n_nodes;  // column blockIdx.y
  xf += blockIdx.y * Lf.n_nodes;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Lf.n_dofs) return;
  const int32_t node = Lf.dof_node[i];
  int J0[3], nq[3];
  double w[3][N1];
  int r = node;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int I = r % Lf.nn;
    r /= Lf.nn;
    const int q = I % (2 * K);
    if (q == 0) { J0[a] = I / 2; nq[a] = 1; w[a][0] = 1.0; }
    else {
      J0[a] = K * (I / (2 * K));
      nq[a] = N1;
#pragma unroll
      for (int bb = 0; bb < N1; ++bb) w[a][bb] = p1d[q * N1 + bb];
    }
  }
  // all (k+1)^d coarse values at once (predicated), then the weighted sum in
  // the order of the contributing combinations
  constexpr int NQ = Pow<N1, D>::v;
  T v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int s0 = q % N1, s1 = (q / N1) % N1, s2 = D == 3 ? q / (N1 * N1) : 0;
    const bool use = s0 < nq[0] && s1 < nq[1] && (D == 2 || s2 < nq[2]);
    int J[3] = {J0[0] + s0, J0[1] + s1, D == 3 ? J0[2] + s2 : 0};
    v[q] = use ? xc[lat(D, Lc.nn, J)] : (T)0;
  }
  T acc = 0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int s0 = q % N1, s1 = (q / N1) % N1, s2 = D == 3 ? q / (N1 * N1) : 0;
    if (s0 < nq[0] && s1 < nq[1] && (D == 2 || s2 < nq[2])) {
      double wt = w[0][s0] * w[1][s1];
      if (D == 3) wt *= w[2][s2];
      acc += (T)wt * v[q];
    }
  }
  xf[node] += acc;
}

template <int D, int K, typename T>
__global__ __launch_bounds__(256) void k_prolong_add(KLevel Lc, KLevel Lf, const T* __restrict__ xc,
                                                     T* __restrict__ xf) {
  prolong_add_body<D, K, T>(Lc, Lf, xc, xf);
}

// argument record of k_prolong_add for grouped launches (k_grouped)
template <int D, int K, typename T>
struct ProlongAddArgs {
  KLevel Lc;
  KLevel Lf;
  const T* xc;
  T* xf;
  __device__ void run() const { prolong_add_body<D, K, T>(Lc, Lf, xc, xf); }
};

// b_c[J] = sum_I P(I, J) r_f[I] for every active coarse node (transpose).  In
// every direction the fine nodes with a non-zero weight form one contiguous
// range: [2J-2k+1, 2J+2k-1] around a coarse vertex, [2kC+1, 2kC+2k-1] inside a
// coarse cell C; the weights are read from the 1-D prolongation table.
template <int K>
__device__ __forceinline__ double restrict_weight(const double* p1d, int J, int I) {
  constexpr int N1 = K + 1;
  if (J % K == 0) {
    const int v = J / K;
    if (I == 2 * J) return 1.0;
    if (I < 2 * J) return p1d[(I - 2 * K * (v - 1)) * N1 + K];
    return p1d[(I - 2 * K * v) * N1 + 0];
  }
  const int C = J / K;
  return p1d[(I - 2 * K * C) * N1 + J % K];
}

template <int D, int K, typename T>
__device__ __forceinline__ void restrict_body(KLevel Lc, KLevel Lf, const T* __restrict__ rf, T* __restrict__ bc) {
  using S = Shape<D, K>;
  constexpr int N1 = S::N1;
  __shared__ double p1d[S::NC1 * N1];
  for (int t = threadIdx.x; t < S::NC1 * N1; t += blockDim.x) p1d[t] = Lf.tables[S::T_P1D + t];
  __syncthreads();
  rf += blockIdx.y * Lf.n_nodes;  // column blockIdx.y
  bc += blockIdx.y * Lc.n_nodes;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= Lc.n_dofs) return;
  const int32_t node = Lc.dof_node[j];
  int J[3], lo[3], hi[3];
  int r = node;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    J[a] = r % Lc.nn;
    r /= Lc.nn;
    if (J[a] % K == 0) {
      lo[a] = 2 * J[a] - 2 * K + 1;
      hi[a] = 2 * J[a] + 2 * K - 1;
    } else {
      const int C = J[a] / K;
      lo[a] = 2 * K * C + 1;
      hi[a] = 2 * K * C + 2 * K - 1;
    }
    lo[a] = lo[a] < 0 ? 0 : lo[a];
    hi[a] = hi[a] > Lf.nn - 1 ? Lf.nn - 1 : hi[a];
  }
  // 1-D weights over the (at most 4k-1 wide) ranges, zero beyond them; the
  // loads of one x-y slab are issued together
  constexpr int WR = 4 * K - 1;
  T w[2][WR];  // directions 0 and 1; direction 2 inside the slab loop (a runtime index)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < WR; ++t) w[a][t] = lo[a] + t <= hi[a] ? (T)restrict_weight<K>(p1d, J[a], lo[a] + t) : (T)0;
  const int64_t nn = Lf.nn;
  T acc = 0;
  for (int t2 = 0; t2 < (D == 3 ? WR : 1); ++t2) {
    if (D == 3 && lo[2] + t2 > hi[2]) break;
    const int64_t base = lo[0] + nn * (lo[1] + (D == 3 ? nn * (lo[2] + t2) : 0));
    T a1 = 0;
    if constexpr (WR * WR * sizeof(T) <= 400) {  // the slab fits in about 100 registers
      T v[WR][WR];
#pragma unroll
      for (int t1 = 0; t1 < WR; ++t1)
#pragma unroll
        for (int t0 = 0; t0 < WR; ++t0)
          v[t1][t0] = (lo[1] + t1 <= hi[1] && lo[0] + t0 <= hi[0]) ? rf[base + t0 + nn * t1] : (T)0;
#pragma unroll
      for (int t1 = 0; t1 < WR; ++t1) {
        if (lo[1] + t1 > hi[1]) continue;
        T a0 = 0;
#pragma unroll
        for (int t0 = 0; t0 < WR; ++t0)
          if (lo[0] + t0 <= hi[0]) a0 += w[0][t0] * v[t1][t0];
        a1 += w[1][t1] * a0;
      }
    } else {  // row by row
      for (int t1 = 0; t1 < WR; ++t1) {
        if (lo[1] + t1 > hi[1]) break;
        T v[WR];
#pragma unroll
        for (int t0 = 0; t0 < WR; ++t0) v[t0] = lo[0] + t0 <= hi[0] ? rf[base + t0 + nn * t1] : (T)0;
        T a0 = 0;
#pragma unroll
        for (int t0 = 0; t0 < WR; ++t0)
          if (lo[0] + t0 <= hi[0]) a0 += w[0][t0] * v[t0];
        a1 += (T)restrict_weight<K>(p1d, J[1], lo[1] + t1) * a0;
      }
    }
    acc += D == 3 ? (T)restrict_weight<K>(p1d, J[2], lo[2] + t2) * a1 : a1;
  }
  bc[node] = acc;
}

template <int D, int K, typename T>
__global__ __launch_bounds__(256) void k_restrict(KLevel Lc, KLevel Lf, const T* __restrict__ rf,
                                                  T* __restrict__ bc) {
  restrict_body<D, K, T>(Lc, Lf, rf, bc);
}

// argument record of k_restrict for grouped launches (k_grouped)
template <int D, int K, typename T>
struct RestrictArgs {
  KLevel Lc;
  KLevel Lf;
  const T* rf;
  T* bc;
  __device__ void run() const { restrict_body<D, K, T>(Lc, Lf, rf, bc); }
};

// x_0 = A_0^{-1} b_0 on the coarsest level: one 64-wide wavefront per row.
template <typename T>
__device__ __forceinline__ void coarse_body(const T* __restrict__ inv, const int32_t* __restrict__ dof_node, int n0,
                                            const T* __restrict__ b, T* __restrict__ x, int64_t ld) {
  const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n0) return;
  b += blockIdx.y * ld;  // column blockIdx.y
  x += blockIdx.y * ld;
  T s = 0;
  for (int j = lane; j < n0; j += 64) s += inv[(int64_t)row * n0 + j] * b[dof_node[j]];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) x[dof_node[row]] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse(const T* __restrict__ inv, const int32_t* __restrict__ dof_node,
                                                int n0, const T* __restrict__ b, T* __restrict__ x, int64_t ld) {
  coarse_body<T>(inv, dof_node, n0, b, x, ld);
}

// argument record of k_coarse for grouped launches (k_grouped)
template <typename T>
struct CoarseArgs {
  const T* inv;
  const int32_t* dof_node;
  int n0;
  const T* b;
  T* x;
  int64_t ld;
  __device__ void run() const { coarse_body<T>(inv, dof_node, n0, b, x, ld); }
};

template <typename T>
__device__ __forceinline__ void zero_active_body(const int32_t* __restrict__ dof_node, int64_t n, T* __restrict__ x,
                                                 int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[blockIdx.y * ld + dof_node[i]] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_active(const int32_t* __restrict__ dof_node, int64_t n,
                                                     T* __restrict__ x, int64_t ld) {
  zero_active_body<T>(dof_node, n, x, ld);
}

// argument record of k_zero_active for grouped launches (k_grouped)
template <typename T>
struct ZeroActiveArgs {
  const int32_t* dof_node;
  int64_t n;
  T* x;
  int64_t ld;
  __device__ void run() const { zero_active_body<T>(dof_node, n, x, ld); }
};

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ dof_node, int64_t n,
                                                 const TS* __restrict__ src, TD* __restrict__ lat_dst, int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) lat_dst[blockIdx.y * ld + dof_node[i]] = (TD)src[blockIdx.y * n + i];
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_gather(const int32_t* __restrict__ dof_node, int64_t n,
                                                const TS* __restrict__ lat_src, TD* __restrict__ dst, int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[blockIdx.y * n + i] = (TD)lat_src[blockIdx.y * ld + dof_node[i]];
}

}  // namespace dev

// ---------------------------------------------------------------------------
// Host launchers: dispatch on (dimension, degree).
namespace {

inline unsigned blocks(int64_t n, int b = 256) { return static_cast<unsigned>((n + b - 1) / b); }

// Launch recorder of the calling thread (see set_launch_recorder).
thread_local std::vector<LaunchRecord>* t_rec = nullptr;

// While recording: append the grouped form of a launch and return true.
template <int LB, typename A>
bool record(dim3 g, dim3 b, const A& a) {
  if (!t_rec) return false;
  LaunchRecord r;
  r.fn = reinterpret_cast<const void*>(&dev::k_grouped<LB, A>);
  r.grid[0] = g.x;
  r.grid[1] = g.y;
  r.block = b.x;
  r.args.assign(reinterpret_cast<const unsigned char*>(&a), reinterpret_cast<const unsigned char*>(&a) + sizeof(A));
  t_rec->push_back(std::move(r));
  return true;
}

// While recording, a launch without a grouped form leaves an empty record
// (the group that recorded it cannot be formed).
bool record_none() {
  if (!t_rec) return false;
  t_rec->push_back(LaunchRecord{});
  return true;
}

// The defaults of LaunchPolicy: a grid cap of 256 CUs x 8 resident 256-thread
// blocks for the grid-stride kernels that stage level tables in LDS (every
// block loads the tables once), and larger blocks for cut-patch launches of
// fewer than 1536 patches (the coarse levels).

template <typename F>
hipError_t dispatch(int d, int k, F&& f) {
  if (d == 2 && k == 1) return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
  if (d == 2 && k == 2) return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
  if (d == 2 && k == 3) return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
  if (d == 3 && k == 1) return f(std::integral_constant<int, 3>{}, std::integral_constant<int, 1>{});
  if (d == 3 && k == 2) return f(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{});
  if (d == 3 && k == 3) return f(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{});
  return hipErrorInvalidValue;
}

}  // namespace

void set_launch_recorder(std::vector<LaunchRecord>* rec) { t_rec = rec; }
bool launch_recording() { return t_rec != nullptr; }

int tables_size(int d, int k) {
  int n = -1;
  (void)dispatch(d, k, [&](auto D, auto K) {
    n = dev::Shape<D.value, K.value>::T_SIZE;
    return hipSuccess;
  });
  return n;
}

template <typename T>
hipError_t launch_apply(int d, int k, const KLevel& L, const T* x, const T* b, T* y, T* W, T* C, hipStream_t s,
                        int ncol, const LaunchPolicy& lp) {
  if (L.n_dofs == 0) return hipSuccess;
  return dispatch(d, k, [&](auto D, auto K) {
    // while recording, the pre-passes are recorded also where they have no
    // work, so that the launch sequence does not depend on the geometry
    if (L.n_faces > 0 || t_rec) {
      const dim3 g(std::max(1u, blocks(L.n_faces)), ncol);
      if (!record<256>(g, dim3(256), dev::FaceWArgs<D.value, K.value, T>{L, x, W})) {
        hipLaunchKernelGGL((dev::k_face_w<D.value, K.value, T>), g, dim3(256), 0, s, L, x, W);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    if (L.n_spec > 0 || t_rec) {
      constexpr int CPB = dev::CellShape<D.value, K.value>::CPB;
      const dim3 g(std::max(1u, static_cast<unsigned>((L.n_spec + CPB - 1) / CPB)));
      if (ncol == 1) {
        if (!record<64>(g, dim3(64), dev::CellAxArgs<D.value, K.value, T, 1>{L, x, W, C, 1}))
          hipLaunchKernelGGL((dev::k_cell_ax<D.value, K.value, T, 1>), g, dim3(64), 0, s, L, x, W, C, 1);
      } else if (!record<64>(g, dim3(64), dev::CellAxArgs<D.value, K.value, T, kMaxCols>{L, x, W, C, ncol})) {
        hipLaunchKernelGGL((dev::k_cell_ax<D.value, K.value, T, kMaxCols>), g, dim3(64), 0, s, L, x, W, C, ncol);
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    // the two tile kernels write disjoint owned nodes
    if (L.n_tiles > 0 || t_rec) {
      const unsigned nb = std::max(1u, std::min<unsigned>(static_cast<unsigned>(L.n_tiles), lp.max_blocks / ncol + 1));
      if (!record<256>(dim3(nb, ncol), dim3(256), dev::ApplyArgs<D.value, K.value, T>{L, x, b, y, C})) {
        hipLaunchKernelGGL((dev::k_apply<D.value, K.value, T>), dim3(nb, ncol), dim3(256), 0, s, L, x, b, y, C);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    if (L.n_tiles_sf > 0 || t_rec) {
      const unsigned nb =
          std::max(1u, std::min<unsigned>(static_cast<unsigned>(L.n_tiles_sf), lp.max_blocks / ncol + 1));
      if (!record<256>(dim3(nb, ncol), dim3(256), dev::ApplySfArgs<D.value, K.value, T>{L, x, b, y})) {
        hipLaunchKernelGGL((dev::k_apply_sf<D.value, K.value, T>), dim3(nb, ncol), dim3(256), 0, s, L, x, b, y);
        return hipGetLastError();
      }
    }
    return hipSuccess;
  });
}

template <typename T>
hipError_t launch_interior_step(int d, int k, const KLevel& L, const int32_t* verts, int nv, T* x, const T* b,
                                hipStream_t s, int ncol, const LaunchPolicy& lp) {
  if (nv == 0 && !t_rec) return hipSuccess;  // recorded also without work (see launch_apply)
  return dispatch(d, k, [&](auto D, auto K) {
    constexpr int PPB = dev::Shape<D.value, K.value>::PPB;
    const unsigned nb = std::max(1u, std::min<unsigned>(blocks(nv, PPB), lp.max_blocks / ncol + 1));
    if (record<256>(dim3(nb, ncol), dim3(256), dev::InteriorStepArgs<D.value, K.value, T>{L, verts, nv, x, b}))
      return hipSuccess;
    hipLaunchKernelGGL((dev::k_interior_step<D.value, K.value, T>), dim3(nb, ncol), dim3(256), 0, s, L, verts, nv,
                       x, b);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_cut_solve(int d, int k, const KLevel& L, const CutGroupDev& G, const T* x, const T* b, T* dbuf,
                            hipStream_t s, int ncol, T* xb, const CopyJob& cj, const LaunchPolicy& lp) {
  if (G.n_patch == 0) return hipSuccess;
  if (record_none()) return hipSuccess;
  return dispatch(d, k, [&](auto D, auto K) {
    using C = dev::CutShape<D.value, K.value>;
    if (xb == nullptr && cj.n != 0) return hipErrorInvalidValue;  // a copy job needs the second buffer
    // small launches (the coarse levels) are bound by the latency of one patch
    // block: twice the threads per patch shortens its serial passes; large
    // ones keep the smaller blocks for occupancy
    auto go = [&](auto th) {
      constexpr int TH = decltype(th)::value;
      CopyJob c2 = cj;
      c2.nblk = static_cast<int>((cj.n + TH * C::COPY - 1) / (TH * C::COPY));
      hipLaunchKernelGGL((dev::k_cut_solve<D.value, K.value, T, TH>), dim3(c2.nblk + G.n_patch, ncol), dim3(TH), 0,
                         s, L, G, x, b, dbuf, xb, c2);
      return hipGetLastError();
    };
    if (C::THREADS < 256 && G.n_patch < lp.small_cut_launch) return go(std::integral_constant<int, 2 * C::THREADS>{});
    return go(std::integral_constant<int, C::THREADS>{});
  });
}

CopyJob cut_copy_job(int d, int k, const CutGroupDev& Gp, int mask) {
  CopyJob cj;
  if (Gp.n_nodes == 0) return cj;
  cj.nodes = Gp.nodes;
  cj.skip = Gp.nxt;
  cj.mask = mask;
  cj.n = Gp.n_nodes;
  (void)d;
  (void)k;
  return cj;  // the launcher sizes the copy blocks for its block size
}

template <typename T>
hipError_t launch_copy_nodes(const int32_t* nodes, int64_t n, const T* src, T* dst, int64_t ld, hipStream_t s,
                             int ncol) {
  if (n == 0) return hipSuccess;
  if (record_none()) return hipSuccess;
  hipLaunchKernelGGL((dev::k_copy_nodes<T>), dim3(blocks(n), ncol), dim3(256), 0, s, nodes, n, src, dst, ld);
  return hipGetLastError();
}

hipError_t launch_cut_solve_mfma(int d, int k, const KLevel& L, const CutGroupDev& G, const float* x, const float* b,
                                 float* W, float* dbuf, int ncol, hipStream_t s) {
  if (G.n_patch == 0) return hipSuccess;
  if (!G.inv_tiles || !G.tile_off || ncol < 1 || ncol > kMaxCols) return hipErrorInvalidValue;
  return dispatch(d, k, [&](auto D, auto K) {
    if (L.n_faces > 0 || t_rec) {  // ghost-face jumps of the current x, all columns
      const dim3 g(std::max(1u, blocks(L.n_faces)), ncol);
      if (!record<256>(g, dim3(256), dev::FaceWArgs<D.value, K.value, float>{L, x, W})) {
        hipLaunchKernelGGL((dev::k_face_w<D.value, K.value, float>), g, dim3(256), 0, s, L, x, W);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    constexpr int TH = dev::CutShape<D.value, K.value>::THREADS;
    if (record<TH>(dim3(G.n_patch), dim3(TH), dev::CutSolveMfmaArgs<D.value, K.value>{L, G, x, b, W, dbuf, ncol}))
      return hipSuccess;
    hipLaunchKernelGGL((dev::k_cut_solve_mfma<D.value, K.value>), dim3(G.n_patch), dim3(TH), 0, s, L, G, x, b, W,
                       dbuf, ncol);
    return hipGetLastError();
  });
}

hipError_t launch_cut_solve_cols(int d, int k, const KLevel& L, const CutGroupDev& G, const double* x,
                                 const double* b, double* W, double* dbuf, int ncol, hipStream_t s) {
  if (G.n_patch == 0) return hipSuccess;
  if (ncol < 1 || ncol > kMaxCols) return hipErrorInvalidValue;
  return dispatch(d, k, [&](auto D, auto K) {
    if (L.n_faces > 0 || t_rec) {  // ghost-face jumps of the current x, all columns
      const dim3 g(std::max(1u, blocks(L.n_faces)), ncol);
      if (!record<256>(g, dim3(256), dev::FaceWArgs<D.value, K.value, double>{L, x, W})) {
        hipLaunchKernelGGL((dev::k_face_w<D.value, K.value, double>), g, dim3(256), 0, s, L, x, W);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    constexpr int TH = dev::CutShape<D.value, K.value>::THREADS;
    if (record<TH>(dim3(G.n_patch), dim3(TH), dev::CutSolveColsArgs<D.value, K.value>{L, G, x, b, W, dbuf, ncol}))
      return hipSuccess;
    hipLaunchKernelGGL((dev::k_cut_solve_cols<D.value, K.value>), dim3(G.n_patch), dim3(TH), 0, s, L, G, x, b, W,
                       dbuf, ncol);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_cut_update(const CutGroupDev& G, const T* dbuf, T* x, int64_t ldx, hipStream_t s, int ncol) {
  if (G.n_nodes == 0) return hipSuccess;
  if (record<256>(dim3(blocks(G.n_nodes), ncol), dim3(256), dev::CutUpdateArgs<T>{G.nodes, G.n_nodes, dbuf, x, ldx}))
    return hipSuccess;
  hipLaunchKernelGGL((dev::k_cut_update<T>), dim3(blocks(G.n_nodes), ncol), dim3(256), 0, s, G.nodes, G.n_nodes, dbuf,
                     x, ldx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(int d, int k, const KLevel& Lc, const KLevel& Lf, const T* xc, T* xf, hipStream_t s,
                              int ncol) {
  return dispatch(d, k, [&](auto D, auto K) {
    if (record<256>(dim3(blocks(Lf.n_dofs), ncol), dim3(256), dev::ProlongAddArgs<D.value, K.value, T>{Lc, Lf, xc, xf}))
      return hipSuccess;
    hipLaunchKernelGGL((dev::k_prolong_add<D.value, K.value, T>), dim3(blocks(Lf.n_dofs), ncol), dim3(256), 0, s, Lc,
                       Lf, xc, xf);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_restrict(int d, int k, const KLevel& Lc, const KLevel& Lf, const T* rf, T* bc, hipStream_t s,
                           int ncol) {
  return dispatch(d, k, [&](auto D, auto K) {
    if (record<256>(dim3(blocks(Lc.n_dofs), ncol), dim3(256), dev::RestrictArgs<D.value, K.value, T>{Lc, Lf, rf, bc}))
      return hipSuccess;
    hipLaunchKernelGGL((dev::k_restrict<D.value, K.value, T>), dim3(blocks(Lc.n_dofs), ncol), dim3(256), 0, s, Lc,
                       Lf, rf, bc);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_coarse(const T* inv, const int32_t* dof_node, int n0, const T* b, T* x, int64_t ld, hipStream_t s,
                         int ncol) {
  if (record<256>(dim3(blocks(n0, 4), ncol), dim3(256), dev::CoarseArgs<T>{inv, dof_node, n0, b, x, ld})) return hipSuccess;
  hipLaunchKernelGGL((dev::k_coarse<T>), dim3(blocks(n0, 4), ncol), dim3(256), 0, s, inv, dof_node, n0, b, x, ld);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zero_active(const int32_t* dof_node, int64_t n, T* x, int64_t ld, hipStream_t s, int ncol) {
  if (n == 0 && !t_rec) return hipSuccess;
  if (record<256>(dim3(std::max(1u, blocks(n)), ncol), dim3(256), dev::ZeroActiveArgs<T>{dof_node, n, x, ld}))
    return hipSuccess;
  hipLaunchKernelGGL((dev::k_zero_active<T>), dim3(blocks(n), ncol), dim3(256), 0, s, dof_node, n, x, ld);
  return hipGetLastError();
}

template <typename TS, typename TD>
hipError_t launch_scatter(const int32_t* dof_node, int64_t n, const TS* src, TD* lat, int64_t ld, hipStream_t s,
                          int ncol) {
  if (n == 0) return hipSuccess;
  if (record_none()) return hipSuccess;
  hipLaunchKernelGGL((dev::k_scatter<TS, TD>), dim3(blocks(n), ncol), dim3(256), 0, s, dof_node, n, src, lat, ld);
  return hipGetLastError();
}

template <typename TS, typename TD>
hipError_t launch_gather(const int32_t* dof_node, int64_t n, const TS* lat, TD* dst, int64_t ld, hipStream_t s,
                         int ncol) {
  if (n == 0) return hipSuccess;
  if (record_none()) return hipSuccess;
  hipLaunchKernelGGL((dev::k_gather<TS, TD>), dim3(blocks(n), ncol), dim3(256), 0, s, dof_node, n, lat, dst, ld);
  return hipGetLastError();
}

#define CMG_INSTANTIATE(T)                                                                                      \
  template hipError_t launch_apply<T>(int, int, const KLevel&, const T*, const T*, T*, T*, T*, hipStream_t, int, \
                                      const LaunchPolicy&);                                                        \
  template hipError_t launch_interior_step<T>(int, int, const KLevel&, const int32_t*, int, T*, const T*,         \
                                              hipStream_t, int, const LaunchPolicy&);                              \
  template hipError_t launch_cut_solve<T>(int, int, const KLevel&, const CutGroupDev&, const T*, const T*, T*,    \
                                          hipStream_t, int, T*, const CopyJob&, const LaunchPolicy&);              \
  template hipError_t launch_copy_nodes<T>(const int32_t*, int64_t, const T*, T*, int64_t, hipStream_t, int);      \
  template hipError_t launch_cut_update<T>(const CutGroupDev&, const T*, T*, int64_t, hipStream_t, int);          \
  template hipError_t launch_prolong_add<T>(int, int, const KLevel&, const KLevel&, const T*, T*, hipStream_t,     \
                                            int);                                                                  \
  template hipError_t launch_restrict<T>(int, int, const KLevel&, const KLevel&, const T*, T*, hipStream_t, int); \
  template hipError_t launch_coarse<T>(const T*, const int32_t*, int, const T*, T*, int64_t, hipStream_t, int);  \
  template hipError_t launch_zero_active<T>(const int32_t*, int64_t, T*, int64_t, hipStream_t, int);
CMG_INSTANTIATE(double)
CMG_INSTANTIATE(float)
template hipError_t launch_scatter<double, double>(const int32_t*, int64_t, const double*, double*, int64_t,
                                                   hipStream_t, int);
template hipError_t launch_gather<double, double>(const int32_t*, int64_t, const double*, double*, int64_t,
                                                  hipStream_t, int);
template hipError_t launch_scatter<double, float>(const int32_t*, int64_t, const double*, float*, int64_t,
                                                  hipStream_t, int);
template hipError_t launch_gather<float, double>(const int32_t*, int64_t, const float*, double*, int64_t,
                                                 hipStream_t, int);

}  // namespace cmg

// ---------------------------------------------------------------------------
// Vector kernels of the Krylov solver on compact vectors.
namespace cmg {
namespace dev {

// Per-block partial sums of x . y (fixed order, so repeat runs are bitwise equal).
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                     int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  x += blockIdx.y * n;  // column blockIdx.y
  y += blockIdx.y * n;
  part += blockIdx.y * gridDim.x;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_axpy(int64_t n, double a, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ __launch_bounds__(256) void k_xpay(int64_t n, double a, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] + a * y[i];
}

// part[j * gridDim.x + blockIdx.x]: partial sums of V_j . w for the rows j =
// blockIdx.y of V (rows of n entries), against one vector w.
__global__ __launch_bounds__(256) void k_rows_dot_partial(const double* __restrict__ V, const double* __restrict__ w,
                                                          int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  V += blockIdx.y * n;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += V[i] * w[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// y += sum_{j < m} c.v[j] V_j (rows of n entries), in increasing j.
__global__ __launch_bounds__(256) void k_rows_combine(int64_t n, int m, RowCoef c, const double* __restrict__ V,
                                                      double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = y[i];
  for (int j = 0; j < m; ++j) acc += c.v[j] * V[j * n + i];
  y[i] = acc;
}

__global__ __launch_bounds__(256) void k_scale(int64_t n, double a, const double* __restrict__ x,
                                               double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// Column-wise forms: column c = blockIdx.y of n entries, coefficient a.v[c].
__global__ __launch_bounds__(256) void k_axpy_cols(int64_t n, ColCoef a, const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t o = blockIdx.y * n;
  if (i < n) y[o + i] += a.v[blockIdx.y] * x[o + i];
}

__global__ __launch_bounds__(256) void k_xpay_cols(int64_t n, ColCoef a, const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t o = blockIdx.y * n;
  if (i < n) y[o + i] = x[o + i] + a.v[blockIdx.y] * y[o + i];
}

}  // namespace dev

hipError_t launch_dot_partial(const double* x, const double* y, int64_t n, double* part, int nblk, hipStream_t s,
                              int ncol) {
  hipLaunchKernelGGL(dev::k_dot_partial, dim3(nblk, ncol), dim3(256), 0, s, x, y, n, part);
  return hipGetLastError();
}

hipError_t launch_rows_dot_partial(const double* V, const double* w, int64_t n, int m, double* part, int nblk,
                                   hipStream_t s) {
  hipLaunchKernelGGL(dev::k_rows_dot_partial, dim3(nblk, m), dim3(256), 0, s, V, w, n, part);
  return hipGetLastError();
}

hipError_t launch_rows_combine(int64_t n, int m, const RowCoef& c, const double* V, double* y, hipStream_t s) {
  if (n == 0 || m == 0) return hipSuccess;
  if (m > kMaxRows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dev::k_rows_combine, dim3((n + 255) / 256), dim3(256), 0, s, n, m, c, V, y);
  return hipGetLastError();
}

hipError_t launch_scale(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_scale, dim3((n + 255) / 256), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(int64_t n, const ColCoef& a, const double* x, double* y, int ncol, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_axpy_cols, dim3((n + 255) / 256, ncol), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_xpay_cols(int64_t n, const ColCoef& a, const double* x, double* y, int ncol, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_xpay_cols, dim3((n + 255) / 256, ncol), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_axpy, dim3((n + 255) / 256), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_xpay(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_xpay, dim3((n + 255) / 256), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

}  // namespace cmg

namespace cmg {
namespace dev {

__global__ __launch_bounds__(256) void k_fill(int64_t n, double v, double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

__global__ __launch_bounds__(256) void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

}  // namespace dev

// The array behind cmg_apply_noalloc.  In host code its name is a host-side
// stand-in, not a device address: the address is taken per device with
// hipGetSymbolAddress and only that address is passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the address is per device: take it with that device current
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_fill(int64_t n, double v, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_fill, dim3((n + 255) / 256), dim3(256), 0, s, n, v, y);
  return hipGetLastError();
}

hipError_t launch_copy(int64_t n, const double* x, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::k_copy, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

}  // namespace cmg

// ---- load vector of Fourier data on the device -----------------------------
namespace cmg {
namespace dev {

__device__ __forceinline__ double rhs_f(const RhsModes& M, int D, const double* x) {
  double v = 0.0;
  for (int q = 0; q < M.n; ++q) {
    double arg = M.phase[q];
    for (int j = 0; j < D; ++j) arg += M_PI * M.kappa[q][j] * x[j];
    v += M.amp[q] * cos(arg);
  }
  return v;
}

template <int K>
__device__ __forceinline__ void rhs_basis(const RhsPlanDev& R, double t, double* psi) {
#pragma unroll
  for (int a = 0; a <= K; ++a) {
    double v = R.coef[a][K];
#pragma unroll
    for (int m = K - 1; m >= 0; --m) v = v * t + R.coef[a][m];
    psi[a] = v;
  }
}

// Cell vectors of the uncut active cells: tensor Gauss rule with k+3 points
// per direction, one thread per cell.
template <int D, int K>
__global__ __launch_bounds__(256) void k_rhs_uncut(RhsPlanDev R, RhsModes M) {
  constexpr int N1 = K + 1, NL = Pow<N1, D>::v, NG = K + 3;
  const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= R.n_uncut) return;
  const int c = R.uncut[u];
  double lo[3];
  {
    int r = c;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      lo[j] = R.lo + (r % R.N) * R.h;
      r /= R.N;
    }
  }
  double hd = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) hd *= R.h;
  double acc[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) acc[a] = 0.0;
  constexpr int NPT = Pow<NG, D>::v;
  for (int p = 0; p < NPT; ++p) {
    double x[3], psi[3][N1], w = hd;
    int r = p;  // the same for every thread: the table loads are scalar
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int m = r % NG;
      r /= NG;
      x[j] = lo[j] + R.h * R.gx[m];
      w *= R.gw[m];
      rhs_basis<K>(R, R.gx[m], psi[j]);
    }
    const double fv = rhs_f(M, D, x) * w;
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      double v = fv;
      int ra = a;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        v *= psi[j][ra % N1];
        ra /= N1;
      }
      acc[a] += v;
    }
  }
  double* out = R.loc + (int64_t)R.act_id[c] * NL;
#pragma unroll
  for (int a = 0; a < NL; ++a) out[a] = acc[a];
}

// Cell vectors of the cut cells: one block per cut cell, thread t takes the
// columns t, t + 256, ... of the cell; along a column only direction e varies,
// so each column sums f w psi_{a_e} per a_e and spreads it with the basis
// factors of the other directions.  The block's partial vectors are reduced
// in a fixed order (butterfly within each wavefront, then the four
// wavefronts in order).
template <int D, int K>
__global__ __launch_bounds__(256) void k_rhs_cut(RhsPlanDev R, RhsModes M) {
  constexpr int N1 = K + 1, NL = Pow<N1, D>::v;
  const int i = blockIdx.x;
  const int c = R.cut[i];
  double lo[3];
  {
    int r = c;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      lo[j] = R.lo + (r % R.N) * R.h;
      r /= R.N;
    }
  }
  double acc[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) acc[a] = 0.0;
  const int64_t c0 = R.col_off[i], c1 = R.col_off[i + 1];
  for (int64_t col = c0 + threadIdx.x; col < c1; col += blockDim.x) {
    const int e = R.ce[col];
    double x[3], psi[3][N1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x[j] = R.cx[j * R.n_col + col];
      rhs_basis<K>(R, (x[j] - lo[j]) / R.h, psi[j]);
    }
    const double w = R.cw[col], t0 = R.ct0[col], t1 = R.ct1[col];
    double ae[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) ae[a] = 0.0;
    for (int t = 0; t < R.nq; ++t) {
      double xt[3];
#pragma unroll
      for (int j = 0; j < D; ++j) xt[j] = j == e ? t0 + (t1 - t0) * R.tx[t] : x[j];
      const double fv = rhs_f(M, D, xt) * w * (t1 - t0) * R.tw[t];
      double pe[N1];
      rhs_basis<K>(R, (xt[e] - lo[e]) / R.h, pe);
#pragma unroll
      for (int a = 0; a < N1; ++a) ae[a] += fv * pe[a];
    }
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      double v = 1.0, s = 0.0;
      int ra = a;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int aj = ra % N1;
        ra /= N1;
        if (j == e) s = ae[aj];
        else v *= psi[j][aj];
      }
      acc[a] += v * s;
    }
  }
  __shared__ double wsum[4][NL];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    double v = acc[a];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) wsum[wave][a] = v;
  }
  __syncthreads();
  if (threadIdx.x < NL) {
    const int a = threadIdx.x;
    R.loc[(int64_t)R.act_id[c] * NL + a] = (wsum[0][a] + wsum[1][a]) + (wsum[2][a] + wsum[3][a]);
  }
}

// b at every DoF: the cell vectors of the (up to 2^d) active cells that
// contain its node, in a fixed order.
template <int D, int K>
__global__ __launch_bounds__(256) void k_rhs_gather(RhsPlanDev R, const int32_t* __restrict__ dof_node,
                                                    int64_t n, double* __restrict__ b) {
  constexpr int N1 = K + 1;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int I[3];
  {
    int r = dof_node[i];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      I[j] = r % R.nn;
      r /= R.nn;
    }
  }
  double v = 0.0;
#pragma unroll
  for (int comb = 0; comb < (1 << D); ++comb) {
    int cell = 0, loc = 0, sc = 1, sl = 1;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sel = (comb >> j) & 1;  // 0: the cell below the node (or the one holding it), 1: above
      int cj, lj;
      if (I[j] % K == 0) {
        cj = I[j] / K - 1 + sel;
        lj = sel ? 0 : K;
      } else {
        ok = ok && sel == 0;
        cj = I[j] / K;
        lj = I[j] % K;
      }
      ok = ok && cj >= 0 && cj < R.N;
      cell += cj * sc;
      loc += lj * sl;
      sc *= R.N;
      sl *= N1;
    }
    if (!ok) continue;
    const int a = R.act_id[cell];
    if (a >= 0) v += R.loc[(int64_t)a * Pow<N1, D>::v + loc];
  }
  b[i] = v;
}

}  // namespace dev

hipError_t launch_rhs_fourier(int d, int k, const RhsPlanDev& R, const RhsModes& M, const int32_t* dof_node,
                              int64_t n_dofs, double* b, hipStream_t s) {
  return dispatch(d, k, [&](auto D, auto K) {
    if (R.n_uncut > 0)
      hipLaunchKernelGGL((dev::k_rhs_uncut<D.value, K.value>), dim3(static_cast<unsigned>((R.n_uncut + 255) / 256)),
                         dim3(256), 0, s, R, M);
    if (R.n_cut > 0)
      hipLaunchKernelGGL((dev::k_rhs_cut<D.value, K.value>), dim3(static_cast<unsigned>(R.n_cut)), dim3(256), 0, s,
                         R, M);
    if (n_dofs > 0)
      hipLaunchKernelGGL((dev::k_rhs_gather<D.value, K.value>), dim3(static_cast<unsigned>((n_dofs + 255) / 256)),
                         dim3(256), 0, s, R, dof_node, n_dofs, b);
    return hipGetLastError();
  });
}

}  // namespace cmg
