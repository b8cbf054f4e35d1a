// C ABI of the CutFEM vertex-patch multigrid: device upload of the hierarchy,
// V-cycle orchestration (paper Section 2.2) and preconditioned CG.
//
// The V-cycle runs in FP64 or, for the mixed-precision preconditioner, in FP32
// (smoother, transfers, level residuals, coarse solve); the FP32 copies of the
// cut-cell matrices and of the local and coarse inverses are rounded from the
// FP64 factorisations.  CG, its operator products and every ABI vector stay
// FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/cutmg.h"
#include "host.h"
#include "kernels.h"

namespace {

thread_local std::string g_last_error;

cmg_status fail(cmg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(...)                                                                                     \
  do {                                                                                                   \
    hipError_t e_ = (__VA_ARGS__);                                                                       \
    if (e_ != hipSuccess) return fail(CMG_EHIP, std::string(#__VA_ARGS__ ": ") + hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)                \
  do {                           \
    cmg_status s_ = (expr);      \
    if (s_ != CMG_OK) return s_; \
  } while (0)

template <typename T>
struct Vecs {
  T* x = nullptr;  // lattice work vectors
  T* b = nullptr;
  T* r = nullptr;
  T* dbuf = nullptr;  // cut-patch corrections of one colour
  T* W = nullptr;     // ghost-face jumps of the operator kernel
  T* C = nullptr;     // special-cell products of the operator kernel
  T* x1 = nullptr;    // second x buffer of the two-buffer cut colour steps
};

struct DevLevel {
  cmg::KLevel kl64{}, kl32{};
  Vecs<double> v64;
  Vecs<float> v32;
  Vecs<double> m64;  // multi-column work vectors (kMaxCols columns), allocated on first use
  Vecs<float> m32;
  int32_t* int_verts[8] = {};
  int n_int[8] = {};
  cmg::CutGroupDev cut64[8] = {}, cut32[8] = {};
  int64_t max_cut_nodes = 0;
  size_t n_w = 0;  // entries of the ghost-face jump buffer
  size_t n_c = 0;  // entries of the special-cell product buffer
  int32_t* region = nullptr;  // cut region (nodes a cut colour step reads)
  int64_t n_region = 0;
};

// Special cells of a level (cut, or with a ghost face) in cell order: their
// background cells, per special cell its cut id and 2d ghost face ids, and per
// cell its special id (-1 active and regular, -2 inactive).
void special_cells(const cmg::HostLevel& h, int dim, std::vector<int32_t>* spec, std::vector<int32_t>* info,
                   std::vector<int32_t>* sid) {
  const int nf = 2 * dim;
  if (sid) sid->assign(static_cast<size_t>(h.n_cells), -2);
  for (int64_t c = 0; c < h.n_cells; ++c) {
    if (!(h.cell_flags[c] & 1)) continue;
    const bool special = h.cut_id[c] >= 0 || h.cell_gid[c] >= 0;
    if (!special) {
      if (sid) (*sid)[c] = -1;
      continue;
    }
    if (sid) (*sid)[c] = static_cast<int32_t>(spec->size());
    spec->push_back(static_cast<int32_t>(c));
    if (!info) continue;
    info->push_back(h.cut_id[c]);
    for (int j = 0; j < nf; ++j)
      info->push_back(h.cell_gid[c] >= 0 ? h.cell_faces[static_cast<size_t>(h.cell_gid[c]) * nf + j] : -1);
  }
}

// The operator tiles (B^d cells, B as in the kernels' tile shape) split by
// what their staged cells -1 .. B-1 hold: all inside the box, active and
// regular (special id -1) -> tsf, the sum-factorised kernel; else -> mix, the
// kernel with dense rows and the special-cell values.
void split_tiles(const cmg::HostLevel& h, int dim, int k, const std::vector<int32_t>& sid,
                 std::vector<int32_t>* mix, std::vector<int32_t>* tsf) {
  const int B = (dim == 3 && k == 3) ? 2 : 4;
  const int NTd = (h.N + B - 1) / B;
  const int ncell = dim == 3 ? (B + 1) * (B + 1) * (B + 1) : (B + 1) * (B + 1);
  for (int32_t t : h.tiles) {
    int tc[3] = {0, 0, 0};
    for (int a = 0, r = t; a < dim; ++a) {
      tc[a] = r % NTd;
      r /= NTd;
    }
    bool regular = true;
    for (int e = 0; e < ncell && regular; ++e) {
      int64_t cl = 0, st = 1;
      for (int a = 0, r = e; a < dim; ++a) {
        const int c = B * tc[a] - 1 + r % (B + 1);
        r /= B + 1;
        if (c < 0 || c >= h.N) regular = false;
        cl += c * st;
        st *= h.N;
      }
      regular = regular && sid[static_cast<size_t>(cl)] == -1;
    }
    (regular ? tsf : mix)->push_back(t);
  }
}

}  // namespace

struct cmg_problem {
  cmg::Hierarchy H;
  std::vector<DevLevel> lv;
  std::vector<void*> owned;
  double* coarse64 = nullptr;
  float* coarse32 = nullptr;
  bool fp32_ready = false;
  bool fp32 = false;  // precision of the V-cycle
  bool m64_ready = false, m32_ready = false, tiles_ready = false;
  // multi-column Krylov vectors (kMaxCols columns of the finest level, compact)
  double *mkr = nullptr, *mkz = nullptr, *mkp = nullptr, *mkq = nullptr, *mpart = nullptr;
  double* mpart_host = nullptr;
  // GMRES basis (restart + 1 rows) and preconditioned basis (restart rows), compact finest level
  double *gV = nullptr, *gZ = nullptr, *gw = nullptr, *gpart = nullptr, *gpart_host = nullptr;
  int g_restart = 0;
  // Krylov vectors (compact, finest level)
  double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr, *part = nullptr;
  double* part_host = nullptr;
  int nblk = 0;
  int device = 0;
  cmg::LaunchPolicy launch;  // block size / grid cap choices by launch size
  int ghost_local = 0;       // cut-patch residuals: 0 exact, 1 patch-local (see cmg_set_ghost_coupling)
  // device quadrature plan of the finest level's load vector (cmg_rhs_fourier_device), on first use
  bool rhs_ready = false;
  cmg::RhsPlanDev rhs{};
  size_t rhs_bytes = 0;
  // kernel timing: launches of the kinds in timing_mask are bracketed by events
  unsigned timing_mask = 0;
  int timing_level = -1;  // -1: every level
  struct Rec {
    int kind, level;
    hipEvent_t a, b;
    int n;  // launches between the two events
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  hipEvent_t done_ev = nullptr;  // see wait_stream
  // V-cycles replayed from captured HIP graphs (see vcycle_graph), keyed by
  // precision, column count and single/multi-column buffers
  // While kernels are timed, a V-cycle is captured in pieces: every run of
  // consecutive timed launches of one kind and level forms a piece of its own,
  // launched between two eagerly recorded events at replay, and the launches
  // between such runs form the others.
  struct Piece {
    hipGraphExec_t exec = nullptr;
    int kind = -1, level = -1;  // kind >= 0: timed launches of one kind and level
    int n = 0;                  // their number
  };
  struct VGraph {
    std::vector<Piece> pieces;
  };
  std::map<int, VGraph> vgraphs;
  bool use_graphs = true;
  bool graphs_broken = false;        // a capture failed: kernel-by-kernel launches from then on
  hipStream_t cap_stream = nullptr;  // capture only; the graphs run on the caller's stream
  hipEvent_t cap_ev = nullptr;       // orders the capture stream with the caller's stream
  struct Capture {
    bool on = false, ok = true;
    int kind = -1, level = -1;       // the piece being captured holds timed launches of this kind and level
    int n = 0;
    std::vector<Piece> pieces;
  } cap;
};

namespace {

template <typename T>
cmg::KLevel& kl(DevLevel& D);
template <>
cmg::KLevel& kl<double>(DevLevel& D) { return D.kl64; }
template <>
cmg::KLevel& kl<float>(DevLevel& D) { return D.kl32; }
template <typename T>
Vecs<T>& vecs(DevLevel& D);
template <>
Vecs<double>& vecs<double>(DevLevel& D) { return D.v64; }
template <>
Vecs<float>& vecs<float>(DevLevel& D) { return D.v32; }
template <typename T>
Vecs<T>& mvecs(DevLevel& D);
template <>
Vecs<double>& mvecs<double>(DevLevel& D) { return D.m64; }
template <>
Vecs<float>& mvecs<float>(DevLevel& D) { return D.m32; }
template <typename T>
cmg::CutGroupDev& cutg(DevLevel& D, int c);
template <>
cmg::CutGroupDev& cutg<double>(DevLevel& D, int c) { return D.cut64[c]; }
template <>
cmg::CutGroupDev& cutg<float>(DevLevel& D, int c) { return D.cut32[c]; }
template <typename T>
T* coarse_inv(cmg_problem* P);
template <>
double* coarse_inv<double>(cmg_problem* P) { return P->coarse64; }
template <>
float* coarse_inv<float>(cmg_problem* P) { return P->coarse32; }

template <typename T>
cmg_status upload(std::vector<void*>& owned, const T* host, size_t n, T** dptr) {
  *dptr = nullptr;
  if (n == 0) return CMG_OK;
  void* p = nullptr;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return fail(CMG_ENOMEM, "device allocation failed");
  owned.push_back(p);
  HIP_TRY(hipMemcpy(p, host, n * sizeof(T), hipMemcpyHostToDevice));
  *dptr = static_cast<T*>(p);
  return CMG_OK;
}

template <typename T>
cmg_status upload(std::vector<void*>& owned, const std::vector<T>& host, T** dptr) {
  return upload(owned, host.data(), host.size(), dptr);
}

cmg_status upload_f32(std::vector<void*>& owned, const std::vector<double>& host, float** dptr) {
  std::vector<float> f(host.begin(), host.end());
  return upload(owned, f, dptr);
}

// Upper triangles (diagonal included, row-major) of n consecutive symmetric
// nl x nl matrices: the cut-cell matrices as the operator's cell pre-pass
// reads them.
template <typename T>
std::vector<T> pack_upper(const std::vector<double>& full, size_t nl) {
  const size_t n = nl == 0 ? 0 : full.size() / (nl * nl);
  std::vector<T> out;
  out.reserve(n * nl * (nl + 1) / 2);
  for (size_t m = 0; m < n; ++m)
    for (size_t a = 0; a < nl; ++a)
      for (size_t b = a; b < nl; ++b) out.push_back(static_cast<T>(full[(m * nl + a) * nl + b]));
  return out;
}

template <typename T>
cmg_status alloc_zero(std::vector<void*>& owned, size_t n, T** dptr) {
  *dptr = nullptr;
  if (n == 0) return CMG_OK;
  void* p = nullptr;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return fail(CMG_ENOMEM, "device allocation failed");
  owned.push_back(p);
  HIP_TRY(hipMemsetAsync(p, 0, n * sizeof(T), nullptr));
  *dptr = static_cast<T*>(p);
  return CMG_OK;
}

// The uploads and zero fills above run on the null stream.  A caller's stream
// created with hipStreamNonBlocking (the serving workers use them) is not
// ordered after the null stream, so every function that allocates on first
// use waits for that work before it returns and kernels on such a stream can
// read the buffers.  Only the null stream is waited for, not other streams.
cmg_status settle() {
  HIP_TRY(hipStreamSynchronize(nullptr));
  return CMG_OK;
}

}  // namespace

// Serialises the library's device allocations, null-stream uploads and
// synchronisations with the capture of V-cycle graphs: a capture in one
// thread (a solve server's worker) and a null-stream copy or device-wide
// synchronisation in another must not overlap.  Recursive: the ensure_*
// helpers call each other.
std::recursive_mutex& cmg::device_mutex() {
  static std::recursive_mutex m;
  return m;
}

namespace {

cmg_status upload_all(cmg_problem* P) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  const cmg::Config& cfg = P->H.cfg;
  const int L = cfg.n_levels;
  auto& own = P->owned;
  P->lv.resize(L);
  for (int l = 0; l < L; ++l) {
    const cmg::HostLevel& h = P->H.levels[l];
    DevLevel& d = P->lv[l];
    cmg::KLevel& k = d.kl64;
    k.N = h.N;
    k.nn = h.nn;
    k.n_dofs = h.n_dofs;
    k.n_nodes = h.n_nodes;
    uint8_t *flags, *ghost;
    int32_t *cut_id, *dn;
    double *cm, *tab;
    TRY(upload(own, h.cell_flags, &flags));
    TRY(upload(own, h.cut_id, &cut_id));
    TRY(upload(own, h.ghost_mask, &ghost));
    TRY(upload(own, h.cut_mats, &cm));
    double* cpk;
    const size_t nl = static_cast<size_t>(std::pow(cfg.k + 1, cfg.dim));
    TRY(upload(own, pack_upper<double>(h.cut_mats, nl), &cpk));
    TRY(upload(own, h.dof_node, &dn));
    const cmg::LevelTables& t = P->H.tables[l];
    std::vector<double> packed;
    for (const auto* v : {&t.kcell, &t.mhat, &t.d0, &t.d1, &t.gcoef, &t.fd_s, &t.fd_dinv, &t.p1d, &t.k1s})
      packed.insert(packed.end(), v->begin(), v->end());
    if (static_cast<int>(packed.size()) != cmg::tables_size(cfg.dim, cfg.k))
      return fail(CMG_EINVAL, "internal: table layout mismatch");
    TRY(upload(own, packed, &tab));
    k.flags = flags;
    k.cut_id = cut_id;
    k.ghost = ghost;
    k.cut_mats = cm;
    k.cut_packed = cpk;
    k.dof_node = dn;
    k.tables = tab;
    k.kcell32 = nullptr;
    int32_t *flow, *cgid, *cfaces, *tiles;
    uint8_t* fdir;
    TRY(upload(own, h.face_lower, &flow));
    TRY(upload(own, h.face_dir, &fdir));
    TRY(upload(own, h.cell_gid, &cgid));
    TRY(upload(own, h.cell_faces, &cfaces));
    k.n_faces = static_cast<int64_t>(h.face_lower.size());
    k.face_lower = flow;
    k.face_dir = fdir;
    k.cell_gid = cgid;
    k.cell_faces = cfaces;
    k.n_cut = h.n_cut;
    {
      std::vector<int32_t> spec, info, sid;
      special_cells(h, cfg.dim, &spec, &info, &sid);
      std::vector<int32_t> tmix, tsf;
      split_tiles(h, cfg.dim, cfg.k, sid, &tmix, &tsf);
      int32_t* dtsf;
      TRY(upload(own, tmix, &tiles));
      TRY(upload(own, tsf, &dtsf));
      k.n_tiles = static_cast<int>(tmix.size());
      k.tiles = tiles;
      k.n_tiles_sf = static_cast<int>(tsf.size());
      k.tiles_sf = dtsf;
      int32_t *dspec, *dinfo, *dsid;
      TRY(upload(own, spec, &dspec));
      TRY(upload(own, info, &dinfo));
      TRY(upload(own, sid, &dsid));
      k.n_spec = static_cast<int64_t>(spec.size());
      k.spec_cells = dspec;
      k.spec_info = dinfo;
      k.cell_sid = dsid;
    }
    d.kl32 = k;
    d.kl32.cut_mats = nullptr;
    d.kl32.cut_packed = nullptr;
    TRY(alloc_zero(own, h.n_nodes, &d.v64.x));
    TRY(alloc_zero(own, h.n_nodes, &d.v64.b));
    TRY(alloc_zero(own, h.n_nodes, &d.v64.r));
    d.n_w = h.face_lower.size() * static_cast<size_t>(cfg.k) * static_cast<size_t>(std::pow(cfg.k + 1, cfg.dim - 1));
    TRY(alloc_zero(own, d.n_w, &d.v64.W));
    d.n_c = static_cast<size_t>(k.n_spec) * static_cast<size_t>(std::pow(cfg.k + 1, cfg.dim));
    TRY(alloc_zero(own, d.n_c, &d.v64.C));
    for (int c = 0; c < 8; ++c) {
      TRY(upload(own, h.int_vertex[c], &d.int_verts[c]));
      d.n_int[c] = static_cast<int>(h.int_vertex[c].size());
      const cmg::CutPatchGroup& g = h.cut[c];
      cmg::CutGroupDev& G = d.cut64[c];
      G.n_patch = static_cast<int>(g.vertex.size());
      G.n_nodes = static_cast<int64_t>(g.nodes.size());
      if (G.n_patch > 0) {
        int32_t *off, *nodes, *vert;
        int64_t* ioff;
        double* inv;
        TRY(upload(own, g.vertex, &vert));
        G.vertex = vert;
        TRY(upload(own, g.off, &off));
        TRY(upload(own, g.inv_off, &ioff));
        TRY(upload(own, g.nodes, &nodes));
        TRY(upload(own, g.inv, &inv));
        G.off = off;
        G.inv_off = ioff;
        G.nodes = nodes;
        G.inv = inv;
        uint8_t* nxt;
        TRY(upload(own, g.nxt, &nxt));
        G.nxt = nxt;
        // the 2^d cells of every patch: cut id and flags | ghost bits << 8
        const int ncell = 1 << cfg.dim, NV = h.N + 1;
        std::vector<int32_t> ccut(static_cast<size_t>(G.n_patch) * ncell, -1);
        std::vector<uint16_t> cfg_bits(static_cast<size_t>(G.n_patch) * ncell, 0);
        for (int q = 0; q < G.n_patch; ++q) {
          int V[3] = {0, 0, 0};
          for (int a = 0, r = g.vertex[q]; a < cfg.dim; ++a) { V[a] = r % NV; r /= NV; }
          for (int o = 0; o < ncell; ++o) {
            int64_t cl = 0, st = 1;
            bool in = true;
            for (int a = 0; a < cfg.dim; ++a) {
              const int c = V[a] - 1 + ((o >> a) & 1);
              in = in && c >= 0 && c < h.N;
              cl += c * st;
              st *= h.N;
            }
            if (!in) continue;
            const size_t e = static_cast<size_t>(q) * ncell + o;
            ccut[e] = h.cut_id[cl];
            cfg_bits[e] = static_cast<uint16_t>(h.cell_flags[cl] | (h.ghost_mask[cl] << 8));
          }
        }
        int32_t* dccut;
        uint16_t* dcfg;
        TRY(upload(own, ccut, &dccut));
        TRY(upload(own, cfg_bits, &dcfg));
        G.cell_cut = dccut;
        G.cell_fg = dcfg;
      }
      d.cut32[c] = G;
      d.cut32[c].inv = nullptr;
      d.max_cut_nodes = std::max(d.max_cut_nodes, G.n_nodes);
    }
    TRY(alloc_zero(own, static_cast<size_t>(d.max_cut_nodes), &d.v64.dbuf));
    TRY(upload(own, h.cut_region, &d.region));
    d.n_region = static_cast<int64_t>(h.cut_region.size());
    if (d.n_region > 0) TRY(alloc_zero(own, h.n_nodes, &d.v64.x1));
  }
  TRY(upload(own, P->H.coarse_inv, &P->coarse64));
  const int64_t n = P->H.levels.back().n_dofs;
  for (double** v : {&P->kr, &P->kz, &P->kp, &P->kq}) TRY(alloc_zero(own, static_cast<size_t>(n), v));
  P->nblk = static_cast<int>(std::min<int64_t>(1024, (n + 255) / 256));
  TRY(alloc_zero(own, static_cast<size_t>(P->nblk), &P->part));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->part_host), P->nblk * sizeof(double), hipHostMallocDefault));
  return settle();
}

// FP32 copies (rounded from the FP64 set-up) and FP32 work vectors, on first use.
cmg_status ensure_fp32(cmg_problem* P) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  if (P->fp32_ready) return CMG_OK;
  auto& own = P->owned;
  for (size_t l = 0; l < P->lv.size(); ++l) {
    const cmg::HostLevel& h = P->H.levels[l];
    DevLevel& d = P->lv[l];
    float* cm;
    TRY(upload_f32(own, h.cut_mats, &cm));
    d.kl32.cut_mats = cm;
    float* cpk;
    const size_t nl = static_cast<size_t>(std::pow(P->H.cfg.k + 1, P->H.cfg.dim));
    TRY(upload(own, pack_upper<float>(h.cut_mats, nl), &cpk));
    d.kl32.cut_packed = cpk;
    float* kc32;
    TRY(upload_f32(own, P->H.tables[l].kcell, &kc32));
    d.kl32.kcell32 = kc32;
    for (int c = 0; c < 8; ++c) {
      if (d.cut32[c].n_patch == 0) continue;
      float* inv;
      TRY(upload_f32(own, h.cut[c].inv, &inv));
      d.cut32[c].inv = inv;
    }
    TRY(alloc_zero(own, h.n_nodes, &d.v32.x));
    TRY(alloc_zero(own, h.n_nodes, &d.v32.b));
    TRY(alloc_zero(own, h.n_nodes, &d.v32.r));
    TRY(alloc_zero(own, d.n_w, &d.v32.W));
    TRY(alloc_zero(own, d.n_c, &d.v32.C));
    TRY(alloc_zero(own, static_cast<size_t>(d.max_cut_nodes), &d.v32.dbuf));
    if (d.n_region > 0) TRY(alloc_zero(own, h.n_nodes, &d.v32.x1));
  }
  TRY(upload_f32(own, P->H.coarse_inv, &P->coarse32));
  TRY(settle());
  P->fp32_ready = true;
  return CMG_OK;
}

// Multi-column work vectors of precision T on every level (kMaxCols columns),
// and the multi-column Krylov vectors, on first use.
template <typename T>
cmg_status ensure_multi(cmg_problem* P) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  bool& ready = std::is_same<T, float>::value ? P->m32_ready : P->m64_ready;
  if (ready) return CMG_OK;
  if (std::is_same<T, float>::value) TRY(ensure_fp32(P));
  auto& own = P->owned;
  const size_t C = cmg::kMaxCols;
  for (size_t l = 0; l < P->lv.size(); ++l) {
    const cmg::HostLevel& h = P->H.levels[l];
    DevLevel& d = P->lv[l];
    Vecs<T>& v = mvecs<T>(d);
    TRY(alloc_zero(own, C * h.n_nodes, &v.x));
    TRY(alloc_zero(own, C * h.n_nodes, &v.b));
    TRY(alloc_zero(own, C * h.n_nodes, &v.r));
    TRY(alloc_zero(own, C * d.n_w, &v.W));
    TRY(alloc_zero(own, C * d.n_c, &v.C));
    TRY(alloc_zero(own, C * static_cast<size_t>(d.max_cut_nodes), &v.dbuf));
    if (d.n_region > 0) TRY(alloc_zero(own, C * h.n_nodes, &v.x1));
  }
  if (!P->mkr) {
    const size_t n = static_cast<size_t>(P->H.levels.back().n_dofs);
    for (double** v : {&P->mkr, &P->mkz, &P->mkp, &P->mkq}) TRY(alloc_zero(own, C * n, v));
    TRY(alloc_zero(own, C * static_cast<size_t>(P->nblk), &P->mpart));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->mpart_host), C * P->nblk * sizeof(double),
                          hipHostMallocDefault));
  }
  TRY(settle());
  ready = true;
  return CMG_OK;
}

// FP32 cut-patch inverses in the tile order of the matrix-core local solve:
// per patch, row blocks of 16 x column blocks of 4, each tile 64 floats with
// lane l = row l%16 + 16 * column l/16, zero beyond the patch size.
cmg_status ensure_tiles(cmg_problem* P) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  if (P->tiles_ready) return CMG_OK;
  TRY(ensure_fp32(P));
  auto& own = P->owned;
  for (size_t l = 0; l < P->lv.size(); ++l) {
    for (int c = 0; c < 8; ++c) {
      const cmg::CutPatchGroup& g = P->H.levels[l].cut[c];
      cmg::CutGroupDev& G = P->lv[l].cut32[c];
      if (G.n_patch == 0) continue;
      std::vector<int64_t> toff(G.n_patch + 1, 0);
      for (int p = 0; p < G.n_patch; ++p) {
        const int64_t nj = g.off[p + 1] - g.off[p];
        toff[p + 1] = toff[p] + ((nj + 15) / 16) * ((nj + 3) / 4) * 64;
      }
      std::vector<float> tiles(static_cast<size_t>(toff[G.n_patch]), 0.f);
      for (int p = 0; p < G.n_patch; ++p) {
        const int nj = g.off[p + 1] - g.off[p];
        const int nrb = (nj + 15) / 16, nkb = (nj + 3) / 4;
        const double* inv = g.inv.data() + g.inv_off[p];
        for (int rb = 0; rb < nrb; ++rb)
          for (int kb = 0; kb < nkb; ++kb)
            for (int ln = 0; ln < 64; ++ln) {
              const int i = rb * 16 + ln % 16, j = kb * 4 + ln / 16;
              if (i < nj && j < nj)
                tiles[toff[p] + (static_cast<int64_t>(rb) * nkb + kb) * 64 + ln] = static_cast<float>(inv[i * nj + j]);
            }
      }
      float* dt;
      int64_t* doff;
      TRY(upload(own, tiles, &dt));
      TRY(upload(own, toff, &doff));
      G.inv_tiles = dt;
      G.tile_off = doff;
    }
  }
  TRY(settle());
  P->tiles_ready = true;
  return CMG_OK;
}

cmg_status check_device(const cmg_problem* p) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (p->lv.empty()) return fail(CMG_EINVAL, "problem was set up on the host only");
  return CMG_OK;
}

cmg_status check_level(const cmg_problem* p, int level, bool need_fine) {
  TRY(check_device(p));
  if (level < (need_fine ? 1 : 0) || level >= p->H.cfg.n_levels) return fail(CMG_EINVAL, "level out of range");
  return CMG_OK;
}

// Ends the capture of the current piece of a V-cycle graph and starts the
// next one (see cmg_problem::Capture); pieces without nodes are dropped.
void cap_cut(cmg_problem* P, bool restart) {
  cmg_problem::Capture& c = P->cap;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(P->cap_stream, &g) != hipSuccess || !g) {
    c.ok = false;
  } else {
    size_t n = 0;
    if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess) c.ok = false;
    if (c.ok && n > 0) {
      cmg_problem::Piece pc;
      pc.kind = c.kind;
      pc.level = c.level;
      pc.n = c.n;
      if (hipGraphInstantiate(&pc.exec, g, nullptr, nullptr, 0) != hipSuccess) c.ok = false;
      else c.pieces.push_back(pc);
    }
    (void)hipGraphDestroy(g);
  }
  if (restart && hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) c.ok = false;
}

// Takes the next two timing events of the pool (which grows when used up).
bool timing_events(cmg_problem* P, hipEvent_t* a, hipEvent_t* b) {
  if (P->pool_used + 2 > P->pool.size()) {
    for (int i = 0; i < 1024; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      P->pool.push_back(e);
    }
  }
  *a = P->pool[P->pool_used++];
  *b = P->pool[P->pool_used++];
  return true;
}

// Brackets one kernel launch with HIP events when its kind is being timed.
// Every launch of a V-cycle capture passes through one: a timed launch opens
// a timed piece (or joins the open one of its kind and level), any other
// launch closes it.
struct KTimer {
  cmg_problem* P;
  hipStream_t s;
  hipEvent_t b = nullptr;
  KTimer(cmg_problem* P_, int kind, int level, hipStream_t s_) : P(P_), s(s_) {
    if (cmg::launch_recording()) return;  // nothing is launched
    const bool timed = (P->timing_mask & (1u << kind)) && (P->timing_level < 0 || level == P->timing_level);
    cmg_problem::Capture& c = P->cap;
    if (c.on) {
      if (!c.ok) return;
      if (timed && c.kind == kind && c.level == level) {
        ++c.n;
      } else if (timed) {
        cap_cut(P, true);
        c.kind = kind;
        c.level = level;
        c.n = 1;
      } else if (c.kind >= 0) {
        cap_cut(P, true);
        c.kind = c.level = -1;
        c.n = 0;
      }
      return;
    }
    if (!timed) return;
    hipEvent_t a;
    if (!timing_events(P, &a, &b)) return;
    (void)hipEventRecord(a, s);
    P->recs.push_back({kind, level, a, b, 1});
  }
  ~KTimer() {
    if (b) (void)hipEventRecord(b, s);
  }
};

enum KernelKind {
  kApply = 0,
  kInterior = 1,
  kCutSolve = 2,
  kCutUpdate = 3,
  kProlong = 4,
  kRestrict = 5,
  kCoarse = 6,
  kLayout = 7,
  kVector = 8
};

// ---- device-side building blocks on the internal lattice vectors ------------
// multi = false: the single-column work vectors (ncol = 1); multi = true: the
// first ncol columns of the multi-column work vectors (kMaxCols columns,
// n_nodes apart), and in FP32 the matrix-core cut-patch solves, whatever ncol
// is, so that a column's result does not depend on how many columns run with it.

template <typename T>
Vecs<T>& work(DevLevel& D, bool multi) {
  return multi ? mvecs<T>(D) : vecs<T>(D);
}

template <typename T>
cmg_status colour_step(cmg_problem* P, int l, bool interior, int colour, hipStream_t s, int ncol = 1,
                       bool multi = false) {
  const int d = P->H.cfg.dim, k = P->H.cfg.k;
  DevLevel& D = P->lv[l];
  Vecs<T>& v = work<T>(D, multi);
  if (interior) {
    // recorded also without patches, so that one lattice shape records one sequence
    if (D.n_int[colour] == 0 && !cmg::launch_recording()) return CMG_OK;
    KTimer t(P, kInterior, l, s);
    HIP_TRY(cmg::launch_interior_step<T>(d, k, kl<T>(D), D.int_verts[colour], D.n_int[colour], v.x, v.b, s, ncol,
                                         P->launch));
    return CMG_OK;
  }
  const cmg::CutGroupDev& G = cutg<T>(D, colour);
  if (G.n_patch == 0) return CMG_OK;
  {
    KTimer t(P, kCutSolve, l, s);
    if constexpr (std::is_same<T, float>::value) {
      if (multi && G.inv_tiles) {
        HIP_TRY(cmg::launch_cut_solve_mfma(d, k, kl<T>(D), G, v.x, v.b, v.W, v.dbuf, ncol, s));
      } else {
        HIP_TRY(cmg::launch_cut_solve<T>(d, k, kl<T>(D), G, v.x, v.b, v.dbuf, s, ncol, nullptr, cmg::CopyJob(),
                                         P->launch));
      }
    } else if (multi) {
      HIP_TRY(cmg::launch_cut_solve_cols(d, k, kl<T>(D), G, v.x, v.b, v.W, v.dbuf, ncol, s));
    } else {
      HIP_TRY(cmg::launch_cut_solve<T>(d, k, kl<T>(D), G, v.x, v.b, v.dbuf, s, ncol, nullptr, cmg::CopyJob(),
                                       P->launch));
    }
  }
  KTimer t(P, kCutUpdate, l, s);
  HIP_TRY(cmg::launch_cut_update<T>(G, v.dbuf, v.x, D.kl64.n_nodes, s, ncol));
  return CMG_OK;
}

// The cut colour steps of one smoothing pass (n_c sweeps over the colours
// that have cut patches; reversed in the post-smoother).  Every step reads x
// as it was at the start of the step (same-coloured patches are updated
// together).  With the single-matrix-row kernel the steps alternate between two
// x buffers: step i reads X[i % 2] and writes X[(i + 1) % 2], where the patch
// blocks store x + d on the colour's internal DoFs and copy blocks bring over
// the previous colour's DoFs that the current colour does not own; X1 is made
// equal to X0 on the cut region first, and an even number of steps ends in
// X0 (an odd last step uses the correction buffer).  The matrix-core kernel
// keeps the correction buffer and a separate update for every step.
template <typename T>
cmg_status cut_steps(cmg_problem* P, int l, bool post, hipStream_t s, int ncol, bool multi) {
  const int d = P->H.cfg.dim, k = P->H.cfg.k;
  DevLevel& D = P->lv[l];
  Vecs<T>& v = work<T>(D, multi);
  const int C = 1 << d;
  std::vector<int> seq;
  for (int r = 0; r < P->H.cfg.n_c; ++r)
    for (int c = 0; c < C; ++c)
      if (cutg<T>(D, c).n_patch > 0) seq.push_back(c);
  if (post) std::reverse(seq.begin(), seq.end());
  // the multi-column kernels (FP32 matrix cores, FP64 all columns per block)
  // write corrections and take the separate update
  bool cols = multi;
  if constexpr (std::is_same<T, float>::value) {
    cols = false;
    for (int c = 0; c < C; ++c) cols = cols || (multi && cutg<T>(D, c).inv_tiles);
  }
  size_t npp = seq.size() - seq.size() % 2;
  if (cols || !v.x1 || npp == 0) npp = 0;
  if (npp > 0) {
    KTimer t(P, kCutUpdate, l, s);
    HIP_TRY(cmg::launch_copy_nodes<T>(D.region, D.n_region, v.x, v.x1, D.kl64.n_nodes, s, ncol));
  }
  T* X[2] = {v.x, v.x1};
  for (size_t i = 0; i < npp; ++i) {
    const cmg::CutGroupDev& G = cutg<T>(D, seq[i]);
    cmg::CopyJob cj;
    if (i > 0) cj = cmg::cut_copy_job(d, k, cutg<T>(D, seq[i - 1]), post ? 2 : 1);
    KTimer t(P, kCutSolve, l, s);
    HIP_TRY(cmg::launch_cut_solve<T>(d, k, kl<T>(D), G, X[i % 2], v.b, v.dbuf, s, ncol, X[(i + 1) % 2], cj,
                                     P->launch));
  }
  for (size_t i = npp; i < seq.size(); ++i) TRY(colour_step<T>(P, l, false, seq[i], s, ncol, multi));
  return CMG_OK;
}

template <typename T>
cmg_status smooth(cmg_problem* P, int l, bool post, hipStream_t s, int ncol = 1, bool multi = false) {
  const int C = 1 << P->H.cfg.dim;
  if (post) TRY(cut_steps<T>(P, l, post, s, ncol, multi));
  for (int i = 0; i < C; ++i) TRY(colour_step<T>(P, l, true, post ? C - 1 - i : i, s, ncol, multi));
  if (!post) TRY(cut_steps<T>(P, l, post, s, ncol, multi));
  return CMG_OK;
}

template <typename T>
cmg_status coarse(cmg_problem* P, hipStream_t s, int ncol = 1, bool multi = false) {
  DevLevel& D = P->lv[0];
  KTimer t(P, kCoarse, 0, s);
  HIP_TRY(cmg::launch_coarse<T>(coarse_inv<T>(P), D.kl64.dof_node, static_cast<int>(P->H.n_coarse),
                                work<T>(D, multi).b, work<T>(D, multi).x, D.kl64.n_nodes, s, ncol));
  return CMG_OK;
}

template <typename T>
cmg_status zero_active(cmg_problem* P, int l, T* x, hipStream_t s, int ncol = 1) {
  KTimer t(P, kLayout, l, s);
  HIP_TRY(cmg::launch_zero_active<T>(P->lv[l].kl64.dof_node, P->lv[l].kl64.n_dofs, x, P->lv[l].kl64.n_nodes, s,
                                     ncol));
  return CMG_OK;
}

template <typename T>
cmg_status apply_lat(cmg_problem* P, int l, const T* x, const T* b, T* y, hipStream_t s, int ncol = 1,
                     bool multi = false) {
  KTimer t(P, kApply, l, s);
  HIP_TRY(cmg::launch_apply<T>(P->H.cfg.dim, P->H.cfg.k, kl<T>(P->lv[l]), x, b, y, work<T>(P->lv[l], multi).W,
                               work<T>(P->lv[l], multi).C, s, ncol, P->launch));
  return CMG_OK;
}

template <typename T>
cmg_status prolong_add(cmg_problem* P, int l, hipStream_t s, int ncol = 1, bool multi = false) {
  KTimer t(P, kProlong, l, s);
  HIP_TRY(cmg::launch_prolong_add<T>(P->H.cfg.dim, P->H.cfg.k, kl<T>(P->lv[l - 1]), kl<T>(P->lv[l]),
                                     work<T>(P->lv[l - 1], multi).x, work<T>(P->lv[l], multi).x, s, ncol));
  return CMG_OK;
}

template <typename T>
cmg_status restrict_(cmg_problem* P, int l, const T* rf, hipStream_t s, int ncol = 1, bool multi = false) {
  KTimer t(P, kRestrict, l, s);
  HIP_TRY(cmg::launch_restrict<T>(P->H.cfg.dim, P->H.cfg.k, kl<T>(P->lv[l - 1]), kl<T>(P->lv[l]), rf,
                                  work<T>(P->lv[l - 1], multi).b, s, ncol));
  return CMG_OK;
}

// V-cycle on the lattice vectors of precision T: x_L = B b_L, zero initial guess.
template <typename T>
cmg_status vcycle_lattice(cmg_problem* P, hipStream_t s, int ncol = 1, bool multi = false) {
  const int L = P->H.cfg.n_levels - 1;
  for (int l = L; l >= 1; --l) {
    Vecs<T>& v = work<T>(P->lv[l], multi);
    TRY(zero_active<T>(P, l, v.x, s, ncol));
    TRY(smooth<T>(P, l, false, s, ncol, multi));
    TRY(apply_lat<T>(P, l, v.x, v.b, v.r, s, ncol, multi));
    TRY(restrict_<T>(P, l, v.r, s, ncol, multi));
  }
  TRY(coarse<T>(P, s, ncol, multi));
  for (int l = 1; l <= L; ++l) {
    TRY(prolong_add<T>(P, l, s, ncol, multi));
    TRY(smooth<T>(P, l, true, s, ncol, multi));
  }
  return CMG_OK;
}

template <typename T>
cmg_status scatter(cmg_problem* P, int l, const double* src, T* lat, hipStream_t s, int ncol = 1) {
  KTimer t(P, kLayout, l, s);
  HIP_TRY(cmg::launch_scatter<double, T>(P->lv[l].kl64.dof_node, P->lv[l].kl64.n_dofs, src, lat,
                                         P->lv[l].kl64.n_nodes, s, ncol));
  return CMG_OK;
}

template <typename T>
cmg_status gather(cmg_problem* P, int l, const T* lat, double* dst, hipStream_t s, int ncol = 1) {
  KTimer t(P, kLayout, l, s);
  HIP_TRY(cmg::launch_gather<T, double>(P->lv[l].kl64.dof_node, P->lv[l].kl64.n_dofs, lat, dst,
                                        P->lv[l].kl64.n_nodes, s, ncol));
  return CMG_OK;
}

// Wait until the work queued on s so far has finished by polling an event
// from this thread: the Krylov loops wait for a reduction every iteration,
// and a blocking stream synchronisation wakes the host up much later than
// the GPU finishes.  A pending query leaves hipErrorNotReady as the thread's
// last error, which is cleared once the event has completed.
cmg_status wait_stream(cmg_problem* P, hipStream_t s) {
  if (!P->done_ev) HIP_TRY(hipEventCreateWithFlags(&P->done_ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(P->done_ev, s));
  for (;;) {
    const hipError_t e = hipEventQuery(P->done_ev);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return fail(CMG_EHIP, hipGetErrorString(e));
  }
  (void)hipGetLastError();
  return CMG_OK;
}

cmg_status dot(cmg_problem* P, const double* x, const double* y, int64_t n, hipStream_t s, double* out) {
  {
    KTimer t(P, kVector, P->H.cfg.n_levels - 1, s);
    HIP_TRY(cmg::launch_dot_partial(x, y, n, P->part, P->nblk, s));
  }
  HIP_TRY(hipMemcpyAsync(P->part_host, P->part, P->nblk * sizeof(double), hipMemcpyDeviceToHost, s));
  TRY(wait_stream(P, s));
  double acc = 0.0;
  for (int i = 0; i < P->nblk; ++i) acc += P->part_host[i];
  *out = acc;
  return CMG_OK;
}

// Column-wise dot products of ncol columns of n entries (multi-column
// buffers): the partial sums and their copy to the host are queued on s, and
// dot_cols_sum adds them up once s has reached that point.
cmg_status dot_cols_start(cmg_problem* P, const double* x, const double* y, int64_t n, int ncol, hipStream_t s) {
  {
    KTimer t(P, kVector, P->H.cfg.n_levels - 1, s);
    HIP_TRY(cmg::launch_dot_partial(x, y, n, P->mpart, P->nblk, s, ncol));
  }
  HIP_TRY(hipMemcpyAsync(P->mpart_host, P->mpart, static_cast<size_t>(ncol) * P->nblk * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  return CMG_OK;
}

void dot_cols_sum(const cmg_problem* P, int ncol, double* out) {
  for (int c = 0; c < ncol; ++c) {
    double acc = 0.0;
    for (int i = 0; i < P->nblk; ++i) acc += P->mpart_host[c * P->nblk + i];
    out[c] = acc;
  }
}

cmg_status dot_cols(cmg_problem* P, const double* x, const double* y, int64_t n, int ncol, hipStream_t s,
                    double* out) {
  TRY(dot_cols_start(P, x, y, n, ncol, s));
  TRY(wait_stream(P, s));
  dot_cols_sum(P, ncol, out);
  return CMG_OK;
}

// V_j . w for the first m rows of the GMRES basis.
cmg_status rows_dot(cmg_problem* P, const double* V, const double* w, int64_t n, int m, hipStream_t s,
                    double* out) {
  {
    KTimer t(P, kVector, P->H.cfg.n_levels - 1, s);
    HIP_TRY(cmg::launch_rows_dot_partial(V, w, n, m, P->gpart, P->nblk, s));
  }
  HIP_TRY(hipMemcpyAsync(P->gpart_host, P->gpart, static_cast<size_t>(m) * P->nblk * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  TRY(wait_stream(P, s));
  for (int j = 0; j < m; ++j) {
    double acc = 0.0;
    for (int i = 0; i < P->nblk; ++i) acc += P->gpart_host[j * P->nblk + i];
    out[j] = acc;
  }
  return CMG_OK;
}

cmg_status ensure_gmres(cmg_problem* P, int restart) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  if (P->g_restart >= restart) return CMG_OK;
  auto& own = P->owned;
  const size_t n = static_cast<size_t>(P->H.levels.back().n_dofs);
  TRY(alloc_zero(own, (restart + 1) * n, &P->gV));
  TRY(alloc_zero(own, restart * n, &P->gZ));
  if (!P->gw) TRY(alloc_zero(own, n, &P->gw));
  TRY(alloc_zero(own, static_cast<size_t>(restart + 1) * P->nblk, &P->gpart));
  if (P->gpart_host) (void)hipHostFree(P->gpart_host);
  P->gpart_host = nullptr;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->gpart_host), (restart + 1) * P->nblk * sizeof(double),
                        hipHostMallocDefault));
  TRY(settle());
  P->g_restart = restart;
  return CMG_OK;
}

// ---- ABI operations in precision T ------------------------------------------

template <typename T>
cmg_status op_apply(cmg_problem* p, int level, const double* x, double* y, hipStream_t s) {
  Vecs<T>& v = vecs<T>(p->lv[level]);
  TRY(scatter<T>(p, level, x, v.x, s));
  TRY(apply_lat<T>(p, level, v.x, nullptr, v.r, s));
  return gather<T>(p, level, v.r, y, s);
}

// The operator product with every intermediate in the per-device scratch
// array instead of the problem's work vectors: lattice x | lattice y | ghost
// face jumps W | special-cell products C, each at a 256-byte boundary.  The
// lattice x is cleared first (its inactive nodes must read zero; the array
// keeps what the previous call left); y, W and C are written in full before
// they are read.  No device or host allocation on the success path (no
// kernel timers either).
template <typename T>
cmg_status op_apply_noalloc(cmg_problem* p, int level, const double* x, double* y, hipStream_t s) {
  DevLevel& D = p->lv[level];
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t nn = static_cast<size_t>(D.kl64.n_nodes);
  const size_t bx = up(nn * sizeof(T)), bw = up(D.n_w * sizeof(T)), bc = up(D.n_c * sizeof(T));
  const size_t need = 2 * bx + bw + bc;
  if (need > cmg::kNoallocScratchBytes)
    return fail(CMG_EINVAL, "level " + std::to_string(level) + " needs " + std::to_string(need) +
                                " bytes of scratch; cmg_apply_noalloc holds at most " +
                                std::to_string(cmg::kNoallocScratchBytes));
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != p->device) return fail(CMG_EINVAL, "cmg_apply_noalloc: the problem lives on another device");
  unsigned char* base = static_cast<unsigned char*>(cmg::noalloc_scratch(cur));
  if (!base) return fail(CMG_EINVAL, "cmg_apply_noalloc: no scratch address for this device (set-up missing)");
  T* xl = reinterpret_cast<T*>(base);
  T* yl = reinterpret_cast<T*>(base + bx);
  T* W = reinterpret_cast<T*>(base + 2 * bx);
  T* C = reinterpret_cast<T*>(base + 2 * bx + bw);
  const int64_t nd = D.kl64.n_dofs, ld = D.kl64.n_nodes;
  HIP_TRY(cmg::launch_fill(static_cast<int64_t>(bx / sizeof(double)), 0.0, reinterpret_cast<double*>(xl), s));
  HIP_TRY(cmg::launch_scatter<double, T>(D.kl64.dof_node, nd, x, xl, ld, s));
  HIP_TRY(cmg::launch_apply<T>(p->H.cfg.dim, p->H.cfg.k, kl<T>(D), xl, static_cast<const T*>(nullptr), yl, W, C, s,
                               1, p->launch));
  HIP_TRY(cmg::launch_gather<T, double>(D.kl64.dof_node, nd, yl, y, ld, s));
  return CMG_OK;
}

template <typename T>
cmg_status op_colour_step(cmg_problem* p, int level, bool interior, int colour, double* x, const double* b,
                          hipStream_t s) {
  Vecs<T>& v = vecs<T>(p->lv[level]);
  TRY(scatter<T>(p, level, x, v.x, s));
  TRY(scatter<T>(p, level, b, v.b, s));
  TRY(colour_step<T>(p, level, interior, colour, s));
  return gather<T>(p, level, v.x, x, s);
}

template <typename T>
cmg_status op_smooth(cmg_problem* p, int level, bool post, double* x, const double* b, hipStream_t s) {
  Vecs<T>& v = vecs<T>(p->lv[level]);
  TRY(scatter<T>(p, level, x, v.x, s));
  TRY(scatter<T>(p, level, b, v.b, s));
  TRY(smooth<T>(p, level, post, s));
  return gather<T>(p, level, v.x, x, s);
}

template <typename T>
cmg_status op_transfer(cmg_problem* p, int level, int dir, const double* x, double* y, hipStream_t s) {
  Vecs<T>& F = vecs<T>(p->lv[level]);
  Vecs<T>& C = vecs<T>(p->lv[level - 1]);
  if (dir == 0) {
    TRY(scatter<T>(p, level - 1, x, C.x, s));
    TRY(zero_active<T>(p, level, F.x, s));
    TRY(prolong_add<T>(p, level, s));
    return gather<T>(p, level, F.x, y, s);
  }
  TRY(scatter<T>(p, level, x, F.r, s));
  TRY(restrict_<T>(p, level, F.r, s));
  return gather<T>(p, level - 1, C.b, y, s);
}

template <typename T>
cmg_status op_coarse(cmg_problem* p, const double* b, double* x, hipStream_t s) {
  Vecs<T>& v = vecs<T>(p->lv[0]);
  TRY(scatter<T>(p, 0, b, v.b, s));
  TRY(coarse<T>(p, s));
  return gather<T>(p, 0, v.x, x, s);
}

void drop_graphs(cmg_problem* P) {
  for (auto& kv : P->vgraphs)
    for (auto& pc : kv.second.pieces) (void)hipGraphExecDestroy(pc.exec);
  P->vgraphs.clear();
}

// The lattice V-cycle as one graph launch on s.  The kernel sequence of a
// V-cycle is fixed for a problem, a precision and a column count, so it is
// captured once (on the problem's own capture stream: the caller's stream may
// be the null stream, which cannot be captured) and replayed: one host call
// instead of ~270 kernel launches, whose host cost otherwise exceeds the GPU
// time of the short coarse-level kernels.  The graph holds kernel nodes only
// (every buffer is cleared by kernels; no memset nodes).  While kernels are
// timed, the timed launches are pieces of their own, bracketed by events
// recorded on s at every replay.  Launch settings, ghost coupling and timing
// changes drop the graphs; a failed capture falls back to kernel-by-kernel
// launches for good.
template <typename T>
cmg_status vcycle_graph(cmg_problem* P, hipStream_t s, int ncol, bool multi) {
  if (!P->use_graphs || P->graphs_broken) return vcycle_lattice<T>(P, s, ncol, multi);
  const int key = (std::is_same<T, float>::value ? 1000 : 0) + (multi ? 100 : 0) + ncol;
  auto it = P->vgraphs.find(key);
  if (it == P->vgraphs.end()) {
    std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
    if (!P->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    if (!P->cap_ev) HIP_TRY(hipEventCreateWithFlags(&P->cap_ev, hipEventDisableTiming));
    // should a capture break off, the launches after it would run on the
    // capture stream: order that stream after s now, and s after it below
    HIP_TRY(hipEventRecord(P->cap_ev, s));
    HIP_TRY(hipStreamWaitEvent(P->cap_stream, P->cap_ev, 0));
    cmg_problem::Capture& c = P->cap;
    c = cmg_problem::Capture{};
    c.on = true;
    if (hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) c.ok = false;
    const cmg_status st = c.ok ? vcycle_lattice<T>(P, P->cap_stream, ncol, multi) : CMG_OK;
    if (c.ok) cap_cut(P, false);
    c.on = false;
    if (st != CMG_OK || !c.ok) {
      // nothing of the capture ran: launch this V-cycle (and all later ones)
      // kernel by kernel
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(P->cap_stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(P->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
      }
      for (auto& pc : c.pieces) (void)hipGraphExecDestroy(pc.exec);
      c.pieces.clear();
      (void)hipGetLastError();
      g_last_error.clear();
      P->graphs_broken = true;
      HIP_TRY(hipEventRecord(P->cap_ev, P->cap_stream));
      HIP_TRY(hipStreamWaitEvent(s, P->cap_ev, 0));
      return vcycle_lattice<T>(P, s, ncol, multi);
    }
    cmg_problem::VGraph g;
    g.pieces = std::move(c.pieces);
    it = P->vgraphs.emplace(key, std::move(g)).first;
  }
  for (const cmg_problem::Piece& pc : it->second.pieces) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool timed = pc.kind >= 0 && timing_events(P, &a, &b);
    if (timed) HIP_TRY(hipEventRecord(a, s));
    HIP_TRY(hipGraphLaunch(pc.exec, s));
    if (timed) {
      HIP_TRY(hipEventRecord(b, s));
      P->recs.push_back({pc.kind, pc.level, a, b, pc.n});
    }
  }
  return CMG_OK;
}

template <typename T>
cmg_status op_vcycle(cmg_problem* p, const double* r, double* z, hipStream_t s) {
  const int L = p->H.cfg.n_levels - 1;
  Vecs<T>& v = vecs<T>(p->lv[L]);
  TRY(scatter<T>(p, L, r, v.b, s));
  TRY(vcycle_graph<T>(p, s, 1, false));
  return gather<T>(p, L, v.x, z, s);
}

cmg_status vcycle_current(cmg_problem* p, const double* r, double* z, hipStream_t s) {
  return p->fp32 ? op_vcycle<float>(p, r, z, s) : op_vcycle<double>(p, r, z, s);
}

// ncol columns: z = B r with the multi-column work vectors (prepared by the caller).
template <typename T>
cmg_status op_vcycle_multi(cmg_problem* p, int ncol, const double* r, double* z, hipStream_t s) {
  const int L = p->H.cfg.n_levels - 1;
  Vecs<T>& v = mvecs<T>(p->lv[L]);
  TRY(scatter<T>(p, L, r, v.b, s, ncol));
  TRY(vcycle_graph<T>(p, s, ncol, true));
  return gather<T>(p, L, v.x, z, s, ncol);
}

cmg_status vcycle_multi_current(cmg_problem* p, int ncol, const double* r, double* z, hipStream_t s) {
  return p->fp32 ? op_vcycle_multi<float>(p, ncol, r, z, s) : op_vcycle_multi<double>(p, ncol, r, z, s);
}

// ncol columns: y = A x in FP64 on the finest level.
cmg_status op_apply_multi(cmg_problem* p, int ncol, const double* x, double* y, hipStream_t s) {
  const int L = p->H.cfg.n_levels - 1;
  Vecs<double>& v = mvecs<double>(p->lv[L]);
  TRY(scatter<double>(p, L, x, v.x, s, ncol));
  TRY(apply_lat<double>(p, L, v.x, nullptr, v.r, s, ncol, true));
  return gather<double>(p, L, v.r, y, s, ncol);
}

cmg_status prepare_multi(cmg_problem* p) {
  TRY(ensure_multi<double>(p));
  if (p->fp32) {
    TRY(ensure_multi<float>(p));
    TRY(ensure_tiles(p));
  }
  return CMG_OK;
}


// Device bytes of a hierarchy once uploaded (see cmg_device_bytes for flags),
// from its counts only: it also serves hierarchies built without the numeric
// part (no cut-cell matrices or inverses), which have every count and size.
size_t hierarchy_bytes(const cmg::Hierarchy& H, int flags) {
  const bool fp32 = flags & 1, multi = flags & 2;
  const cmg::Config& cfg = H.cfg;
  const size_t nt = static_cast<size_t>(cmg::tables_size(cfg.dim, cfg.k));
  const size_t nw_face = static_cast<size_t>(cfg.k) * static_cast<size_t>(std::pow(cfg.k + 1, cfg.dim - 1));
  const size_t nl = static_cast<size_t>(std::pow(cfg.k + 1, cfg.dim));
  const size_t C = cmg::kMaxCols;
  size_t b64 = 0, b32 = 0, m64 = 0, m32 = 0;
  for (const cmg::HostLevel& h : H.levels) {
    size_t maxn = 0;
    // cut-cell matrix entries: full (rows of the cut steps) and packed upper triangles (operator)
    const size_t ncm = static_cast<size_t>(h.n_cut) * (nl * nl + nl * (nl + 1) / 2);
    b64 += h.cell_flags.size() + h.ghost_mask.size() + 4 * (h.cut_id.size() + h.dof_node.size()) +
           8 * (ncm + nt) + 4 * (h.face_lower.size() + h.cell_gid.size() + h.cell_faces.size() +
           h.tiles.size()) + h.face_dir.size();
    b64 += 8 * (3 * static_cast<size_t>(h.n_nodes) + h.face_lower.size() * nw_face);
    b32 += 4 * (ncm + nl * nl + 3 * static_cast<size_t>(h.n_nodes) + h.face_lower.size() * nw_face);
    for (int c = 0; c < 8; ++c) {
      const cmg::CutPatchGroup& g = h.cut[c];
      const size_t ninv = g.inv_off.empty() ? 0 : static_cast<size_t>(g.inv_off.back());
      b64 += 4 * (h.int_vertex[c].size() + g.vertex.size() + g.off.size() + g.nodes.size()) + 8 * g.inv_off.size() +
             8 * ninv + g.nxt.size() + 6 * g.vertex.size() * (size_t{1} << cfg.dim);
      b32 += 4 * ninv;
      maxn = std::max(maxn, g.nodes.size());
      if (g.vertex.empty()) continue;
      m32 += 8 * (g.vertex.size() + 1);  // tile offsets
      for (size_t q = 0; q + 1 < g.off.size(); ++q) {
        const size_t nj = static_cast<size_t>(g.off[q + 1] - g.off[q]);
        m32 += 4 * ((nj + 15) / 16) * ((nj + 3) / 4) * 64;
      }
    }
    b64 += 8 * maxn;
    b32 += 4 * maxn;
    std::vector<int32_t> spec;
    special_cells(h, cfg.dim, &spec, nullptr, nullptr);
    const size_t ncc = spec.size() * nl;
    b64 += 8 * ncc;  // special-cell products of the operator
    b32 += 4 * ncc;
    b64 += 4 * (spec.size() * (2 + 2 * cfg.dim) + static_cast<size_t>(h.n_cells));  // special-cell lists
    const size_t nx1 = h.cut_region.empty() ? 0 : static_cast<size_t>(h.n_nodes);  // second x buffer
    b64 += 4 * h.cut_region.size() + 8 * nx1;
    b32 += 4 * nx1;
    const size_t per_col = 3 * static_cast<size_t>(h.n_nodes) + h.face_lower.size() * nw_face + maxn + ncc + nx1;
    m64 += 8 * C * per_col;
    m32 += 4 * C * per_col;
  }
  const size_t nL = static_cast<size_t>(H.levels.back().n_dofs);
  const size_t n0sq = static_cast<size_t>(H.n_coarse) * static_cast<size_t>(H.n_coarse);
  b64 += 8 * n0sq + 8 * 4 * nL + 8 * 1024;
  b32 += 4 * n0sq;
  m64 += 8 * 4 * C * nL + 8 * C * 1024;
  return b64 + (fp32 ? b32 : 0) + (multi ? m64 + (fp32 ? m32 : 0) : 0);
}

}  // namespace

// Grouped V-cycles: the same V-cycle step of every member as one launch.
struct cmg_group {
  std::vector<cmg_problem*> m;
  bool fp32 = false;
  struct Step {
    const void* fn;  // grouped kernel
    dim3 grid;       // largest member grid, z = members
    dim3 block;
    size_t off;      // the members' argument records in tab
  };
  std::vector<Step> steps;
  unsigned char* tab = nullptr;  // device: argument records, one array per step
  bool use_graph = true;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  hipEvent_t cap_ev = nullptr;
};

namespace {

constexpr int kMaxGroup = 8;

void group_release(cmg_group* g) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  if (g->tab || g->exec) (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->cap_ev) (void)hipEventDestroy(g->cap_ev);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->tab) (void)hipFree(g->tab);
  g->exec = nullptr;
  g->cap_ev = nullptr;
  g->cap_stream = nullptr;
  g->tab = nullptr;
}

// Records every member's lattice V-cycle (the multi-column form with one
// column), checks that the members' launch sequences match step by step and
// uploads the argument records.
template <typename T>
cmg_status group_plan(cmg_group* g) {
  const size_t G = g->m.size();
  std::vector<std::vector<cmg::LaunchRecord>> rec(G);
  for (size_t i = 0; i < G; ++i) {
    cmg::set_launch_recorder(&rec[i]);
    const cmg_status st = vcycle_lattice<T>(g->m[i], nullptr, 1, true);
    cmg::set_launch_recorder(nullptr);
    TRY(st);
  }
  const size_t ns = rec[0].size();
  size_t bytes = 0;
  for (size_t i = 1; i < G; ++i)
    if (rec[i].size() != ns)
      return fail(CMG_EINVAL, "group members differ in their V-cycle steps (member " + std::to_string(i) + ")");
  for (size_t j = 0; j < ns; ++j) {
    const cmg::LaunchRecord& r0 = rec[0][j];
    cmg_group::Step st{r0.fn, dim3(0, 0, static_cast<unsigned>(G)), dim3(r0.block), bytes};
    for (size_t i = 0; i < G; ++i) {
      const cmg::LaunchRecord& r = rec[i][j];
      if (!r.fn || r.fn != r0.fn || r.block != r0.block || r.args.size() != r0.args.size())
        return fail(CMG_EINVAL, "group members differ in V-cycle step " + std::to_string(j) + " (member " +
                                    std::to_string(i) + ")");
      st.grid.x = std::max(st.grid.x, r.grid[0]);
      st.grid.y = std::max(st.grid.y, r.grid[1]);
    }
    g->steps.push_back(st);
    bytes += (G * r0.args.size() + 255) / 256 * 256;
  }
  std::vector<unsigned char> host(bytes);
  for (size_t j = 0; j < ns; ++j)
    for (size_t i = 0; i < G; ++i) {
      const std::vector<unsigned char>& a = rec[i][j].args;
      std::memcpy(host.data() + g->steps[j].off + i * a.size(), a.data(), a.size());
    }
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  HIP_TRY(hipMalloc(&g->tab, bytes));
  HIP_TRY(hipMemcpy(g->tab, host.data(), bytes, hipMemcpyHostToDevice));
  return settle();
}

hipError_t group_launch(cmg_group* g, hipStream_t s) {
  for (const cmg_group::Step& st : g->steps) {
    void* a = g->tab + st.off;
    void* args[] = {&a};
    const hipError_t e = hipLaunchKernel(st.fn, st.grid, st.block, args, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The grouped lattice V-cycle, replayed from a graph captured at its first run
// (launched step by step if the capture fails).
cmg_status group_lattice(cmg_group* g, hipStream_t s) {
  if (g->use_graph && !g->exec) {
    std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
    if (!g->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    if (!g->cap_ev) HIP_TRY(hipEventCreateWithFlags(&g->cap_ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(g->cap_ev, s));
    HIP_TRY(hipStreamWaitEvent(g->cap_stream, g->cap_ev, 0));
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      ok = group_launch(g, g->cap_stream) == hipSuccess;
      ok = hipStreamEndCapture(g->cap_stream, &graph) == hipSuccess && ok && graph;
    }
    if (ok) ok = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
      // nothing of the capture ran: launch step by step from now on
      g->exec = nullptr;
      g->use_graph = false;
      (void)hipGetLastError();
    }
    HIP_TRY(hipEventRecord(g->cap_ev, g->cap_stream));
    HIP_TRY(hipStreamWaitEvent(s, g->cap_ev, 0));
  }
  if (g->exec) {
    HIP_TRY(hipGraphLaunch(g->exec, s));
  } else {
    HIP_TRY(group_launch(g, s));
  }
  return CMG_OK;
}

// z[m] = B_m r[m] for every member, in the precision of the group: the steps of
// op_vcycle_multi with one column, the lattice V-cycle grouped.
template <typename T>
cmg_status group_vcycle_t(cmg_group* g, const double* const* r, double* const* z, hipStream_t s) {
  for (size_t i = 0; i < g->m.size(); ++i) {
    cmg_problem* p = g->m[i];
    const int L = p->H.cfg.n_levels - 1;
    TRY(scatter<T>(p, L, r[i], mvecs<T>(p->lv[L]).b, s, 1));
  }
  TRY(group_lattice(g, s));
  for (size_t i = 0; i < g->m.size(); ++i) {
    cmg_problem* p = g->m[i];
    const int L = p->H.cfg.n_levels - 1;
    TRY(gather<T>(p, L, mvecs<T>(p->lv[L]).x, z[i], s, 1));
  }
  return CMG_OK;
}

cmg_status group_vcycle(cmg_group* g, const double* const* r, double* const* z, hipStream_t s) {
  return g->fp32 ? group_vcycle_t<float>(g, r, z, s) : group_vcycle_t<double>(g, r, z, s);
}

}  // namespace

extern "C" {

const char* cmg_last_error(void) { return g_last_error.c_str(); }

// Checks the level set and the parameters and fills the host configuration.
static cmg_status make_config(const cmg_levelset* ls, const cmg_params* prm, cmg::Config* out) {
  if (!ls || !prm) return fail(CMG_EINVAL, "null argument");
  if (ls->dim < 2 || ls->dim > 3 || ls->n_shapes < 1 || !ls->centers || !ls->semi || !(ls->box_hi > ls->box_lo))
    return fail(CMG_EINVAL, "bad level set description");
  if (prm->k < 1 || prm->k > 3 || prm->n_levels < 1 || prm->n_levels > 12 || prm->coarse_cells < 1 ||
      prm->n_c < 0 || prm->quad_n < 2 || prm->quad_n > 64 || prm->ghost_exp_mode < 0 || prm->ghost_exp_mode > 1 ||
      prm->precond_fp32 < 0 || prm->precond_fp32 > 1)
    return fail(CMG_EINVAL, "bad parameters");
  const int64_t fine = static_cast<int64_t>(prm->coarse_cells) << (prm->n_levels - 1);
  if (std::pow(static_cast<double>(prm->k * fine + 1), ls->dim) > 2.0e9)
    return fail(CMG_EINVAL, "lattice too large for 32-bit node indices");
  cmg::Config cfg;
  cfg.dim = ls->dim;
  cfg.k = prm->k;
  cfg.n_levels = prm->n_levels;
  cfg.coarse_cells = prm->coarse_cells;
  cfg.lo = ls->box_lo;
  cfg.hi = ls->box_hi;
  for (int i = 0; i < ls->n_shapes; ++i) {
    cmg::Shape sh;
    for (int j = 0; j < ls->dim; ++j) {
      sh.c[j] = ls->centers[i * ls->dim + j];
      sh.s[j] = ls->semi[i * ls->dim + j];
      if (!(sh.s[j] > 0.0)) return fail(CMG_EINVAL, "semi-axes must be positive");
    }
    cfg.shapes.push_back(sh);
  }
  if (cfg.shapes.size() > 16) return fail(CMG_EINVAL, "at most 16 shapes");
  cfg.gamma_D = prm->gamma_D;
  cfg.gamma_g = prm->gamma_g;
  for (int m = 0; m < 3; ++m) cfg.gamma_m[m] = prm->gamma_m[m];
  cfg.ghost_exp_mode = prm->ghost_exp_mode;
  cfg.n_c = prm->n_c;
  cfg.quad_n = prm->quad_n;
  *out = cfg;
  return CMG_OK;
}

static cmg_status hierarchy_status(const std::string& err) {
  cmg_status st = CMG_EINVAL;
  if (err.rfind("EGEOM", 0) == 0) st = CMG_EGEOM;
  if (err.rfind("ENOTSPD", 0) == 0) st = CMG_ENOTSPD;
  return fail(st, err);
}

static cmg_status setup_impl(const cmg_levelset* ls, const cmg_params* prm, cmg_problem** out, bool device) {
  g_last_error.clear();
  if (!out) return fail(CMG_EINVAL, "null argument");
  *out = nullptr;
  cmg::Config cfg;
  TRY(make_config(ls, prm, &cfg));
  auto* P = new cmg_problem();
  std::string err = cmg::build_hierarchy(cfg, P->H);
  if (!err.empty()) {
    delete P;
    return hierarchy_status(err);
  }
  if (!device) {
    P->fp32 = prm->precond_fp32 != 0;
    *out = P;
    return CMG_OK;
  }
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return fail(CMG_EHIP, "no HIP device");
  }
  std::unique_lock<std::recursive_mutex> lock(cmg::device_mutex());
  cmg_status st = upload_all(P);
  if (st == CMG_OK && cmg::noalloc_scratch_init(P->device) != hipSuccess)
    st = fail(CMG_EHIP, "device address of the allocation-free scratch");
  if (st == CMG_OK && prm->precond_fp32) {
    st = ensure_fp32(P);
    P->fp32 = true;
  }
  if (st != CMG_OK) {
    std::string msg = g_last_error;
    cmg_destroy(P);
    return fail(st, msg);
  }
  *out = P;
  return CMG_OK;
}

cmg_status cmg_setup(const cmg_levelset* ls, const cmg_params* prm, cmg_problem** out) {
  return setup_impl(ls, prm, out, true);
}

cmg_status cmg_setup_host(const cmg_levelset* ls, const cmg_params* prm, cmg_problem** out) {
  return setup_impl(ls, prm, out, false);
}

void cmg_destroy(cmg_problem* p) {
  if (!p) return;
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  if (!p->lv.empty()) (void)hipDeviceSynchronize();
  for (void* v : p->owned) (void)hipFree(v);
  if (p->part_host) (void)hipHostFree(p->part_host);
  if (p->mpart_host) (void)hipHostFree(p->mpart_host);
  if (p->gpart_host) (void)hipHostFree(p->gpart_host);
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  if (p->done_ev) (void)hipEventDestroy(p->done_ev);
  drop_graphs(p);
  if (p->cap_ev) (void)hipEventDestroy(p->cap_ev);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

cmg_status cmg_upload(cmg_problem* p) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (!p->lv.empty()) return CMG_OK;
  if (hipGetDevice(&p->device) != hipSuccess) return fail(CMG_EHIP, "no HIP device");
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  cmg_status st = upload_all(p);
  if (st == CMG_OK && cmg::noalloc_scratch_init(p->device) != hipSuccess)
    st = fail(CMG_EHIP, "device address of the allocation-free scratch");
  if (st == CMG_OK && p->fp32) st = ensure_fp32(p);
  return st;
}

cmg_status cmg_device_bytes(const cmg_problem* p, int flags, size_t* bytes) {
  if (!p || !bytes) return fail(CMG_EINVAL, "null argument");
  if (flags < 0 || flags > 7)
    return fail(CMG_EINVAL, "flags: bit 0 FP32 copies, bit 1 multi-column buffers, bit 2 load-vector plan");
  *bytes = hierarchy_bytes(p->H, flags & 3) + ((flags & 4) && p->rhs_ready ? p->rhs_bytes : 0);
  return CMG_OK;
}

cmg_status cmg_footprint(const cmg_levelset* ls, const cmg_params* prm, int flags, size_t* bytes,
                         int64_t* n_dofs) {
  g_last_error.clear();
  if (!bytes) return fail(CMG_EINVAL, "null argument");
  if (flags < 0 || flags > 3) return fail(CMG_EINVAL, "flags: bit 0 FP32 copies, bit 1 multi-column buffers");
  cmg::Config cfg;
  TRY(make_config(ls, prm, &cfg));
  cmg::Hierarchy H;
  const std::string err = cmg::build_hierarchy(cfg, H, false);
  if (!err.empty()) return hierarchy_status(err);
  *bytes = hierarchy_bytes(H, flags);
  if (n_dofs) *n_dofs = H.levels.back().n_dofs;
  return CMG_OK;
}

cmg_status cmg_set_launch(cmg_problem* p, int small_cut_launch, int max_blocks) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (small_cut_launch < 0 || max_blocks < 1) return fail(CMG_EINVAL, "bad launch policy");
  p->launch.small_cut_launch = small_cut_launch;
  p->launch.max_blocks = static_cast<unsigned>(max_blocks);
  drop_graphs(p);
  return CMG_OK;
}

// Quadrature plan of the device load vector: built on the host (the cut
// cells' columns, OpenMP) and uploaded on the first call.  Synchronous.
static cmg_status ensure_rhs_plan(cmg_problem* P) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  if (P->rhs_ready) return CMG_OK;
  const cmg::Config& cfg = P->H.cfg;
  const cmg::HostLevel& L = P->H.levels.back();
  cmg::RhsPlan R;
  cmg::build_rhs_plan(P->H, R);
  cmg::RhsPlanDev& D = P->rhs;
  D = cmg::RhsPlanDev{};
  D.N = L.N;
  D.nn = L.nn;
  D.lo = cfg.lo;
  D.h = L.h;
  D.n_uncut = static_cast<int64_t>(R.uncut.size());
  D.n_cut = static_cast<int64_t>(R.cut.size());
  D.n_col = static_cast<int64_t>(R.cw.size());
  auto& own = P->owned;
  int32_t *uncut, *cut, *act;
  int64_t* off;
  double *cx, *cw, *ct0, *ct1, *loc;
  uint8_t* ce;
  TRY(upload(own, R.uncut, &uncut));
  TRY(upload(own, R.cut, &cut));
  TRY(upload(own, R.col_off, &off));
  TRY(upload(own, R.cx, &cx));
  TRY(upload(own, R.cw, &cw));
  TRY(upload(own, R.ct0, &ct0));
  TRY(upload(own, R.ct1, &ct1));
  TRY(upload(own, R.ce, &ce));
  TRY(upload(own, R.act_id, &act));
  const int nl = static_cast<int>(std::pow(cfg.k + 1, cfg.dim));
  TRY(alloc_zero(own, static_cast<size_t>(R.n_active) * nl, &loc));
  TRY(settle());
  D.uncut = uncut;
  D.cut = cut;
  D.col_off = off;
  D.cx = cx;
  D.cw = cw;
  D.ct0 = ct0;
  D.ct1 = ct1;
  D.ce = ce;
  D.act_id = act;
  D.loc = loc;
  for (int a = 0; a <= cfg.k; ++a)
    for (int m = 0; m <= cfg.k; ++m) D.coef[a][m] = P->H.basis.coef[a][m];
  cmg::gauss_legendre(cfg.k + 3, D.gx, D.gw);
  D.nq = cfg.quad_n;
  cmg::gauss_legendre(cfg.quad_n, D.tx, D.tw);
  P->rhs_bytes = R.uncut.size() * 4 + R.cut.size() * 4 + R.col_off.size() * 8 + R.cx.size() * 8 +
                 R.cw.size() * 24 + R.ce.size() + R.act_id.size() * 4 + static_cast<size_t>(R.n_active) * nl * 8;
  P->rhs_ready = true;
  return CMG_OK;
}

cmg_status cmg_rhs_fourier_device(cmg_problem* p, int n_modes, const int* kappa, const double* amp,
                                  const double* phase, double* b, void* stream) {
  TRY(check_device(p));
  if (!b || n_modes < 0 || n_modes > cmg::kMaxModes || (n_modes > 0 && (!kappa || !amp || !phase)))
    return fail(CMG_EINVAL, "bad Fourier right-hand side (at most 32 modes)");
  if (p->H.cfg.quad_n > 16) return fail(CMG_EINVAL, "the device load vector takes at most 16 points per piece");
  TRY(ensure_rhs_plan(p));
  cmg::RhsModes M{};
  M.n = n_modes;
  const int d = p->H.cfg.dim;
  for (int q = 0; q < n_modes; ++q) {
    for (int j = 0; j < d; ++j) M.kappa[q][j] = kappa[q * d + j];
    M.amp[q] = amp[q];
    M.phase[q] = phase[q];
  }
  const cmg::HostLevel& L = p->H.levels.back();
  DevLevel& D = p->lv.back();
  HIP_TRY(cmg::launch_rhs_fourier(d, p->H.cfg.k, p->rhs, M, D.kl64.dof_node, L.n_dofs, b,
                                  static_cast<hipStream_t>(stream)));
  return CMG_OK;
}

cmg_status cmg_apply_noalloc(cmg_problem* p, int level, const double* x, double* y, void* stream) {
  TRY(check_level(p, level, false));
  if (!x || !y) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  return p->fp32 ? op_apply_noalloc<float>(p, level, x, y, s) : op_apply_noalloc<double>(p, level, x, y, s);
}

cmg_status cmg_set_ghost_coupling(cmg_problem* p, int mode) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (mode != 0 && mode != 1) return fail(CMG_EINVAL, "ghost coupling mode must be 0 or 1");
  p->ghost_local = mode;
  for (DevLevel& d : p->lv) {
    d.kl64.ghost_local = mode;
    d.kl32.ghost_local = mode;
  }
  drop_graphs(p);
  return CMG_OK;
}

cmg_status cmg_set_graphs(cmg_problem* p, int enable) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (enable != 0 && enable != 1) return fail(CMG_EINVAL, "graph flag must be 0 or 1");
  p->use_graphs = enable != 0;
  drop_graphs(p);
  return CMG_OK;
}

cmg_status cmg_set_precision(cmg_problem* p, int fp32) {
  TRY(check_device(p));
  if (fp32 != 0 && fp32 != 1) return fail(CMG_EINVAL, "precision flag must be 0 or 1");
  if (fp32) TRY(ensure_fp32(p));
  p->fp32 = fp32 != 0;
  return CMG_OK;
}

cmg_status cmg_ndofs(const cmg_problem* p, int level, int64_t* n) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (level < 0 || level >= p->H.cfg.n_levels) return fail(CMG_EINVAL, "level out of range");
  if (!n) return fail(CMG_EINVAL, "null output");
  *n = p->H.levels[level].n_dofs;
  return CMG_OK;
}

cmg_status cmg_apply(cmg_problem* p, int level, const double* x, double* y, void* stream) {
  TRY(check_level(p, level, false));
  if (!x || !y) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  return p->fp32 ? op_apply<float>(p, level, x, y, s) : op_apply<double>(p, level, x, y, s);
}

cmg_status cmg_colour_step(cmg_problem* p, int level, int interior, int colour, double* x, const double* b,
                           void* stream) {
  TRY(check_level(p, level, true));
  if (colour < 0 || colour >= (1 << p->H.cfg.dim)) return fail(CMG_EINVAL, "colour out of range");
  if (!x || !b) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  return p->fp32 ? op_colour_step<float>(p, level, interior != 0, colour, x, b, s)
                 : op_colour_step<double>(p, level, interior != 0, colour, x, b, s);
}

cmg_status cmg_smooth(cmg_problem* p, int level, int post, double* x, const double* b, void* stream) {
  TRY(check_level(p, level, true));
  if (!x || !b) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  return p->fp32 ? op_smooth<float>(p, level, post != 0, x, b, s) : op_smooth<double>(p, level, post != 0, x, b, s);
}

cmg_status cmg_transfer(cmg_problem* p, int level, int dir, const double* x, double* y, void* stream) {
  TRY(check_level(p, level, true));
  if (!x || !y || (dir != 0 && dir != 1)) return fail(CMG_EINVAL, "bad transfer arguments");
  auto s = static_cast<hipStream_t>(stream);
  return p->fp32 ? op_transfer<float>(p, level, dir, x, y, s) : op_transfer<double>(p, level, dir, x, y, s);
}

cmg_status cmg_coarse_solve(cmg_problem* p, const double* b, double* x, void* stream) {
  TRY(check_device(p));
  if (!x || !b) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  return p->fp32 ? op_coarse<float>(p, b, x, s) : op_coarse<double>(p, b, x, s);
}

cmg_status cmg_vcycle(cmg_problem* p, const double* r, double* z, void* stream) {
  TRY(check_device(p));
  if (!r || !z) return fail(CMG_EINVAL, "null argument");
  return vcycle_current(p, r, z, static_cast<hipStream_t>(stream));
}

cmg_status cmg_solve(cmg_problem* p, const double* b, double* x, double rtol, int maxit, cmg_solve_info* info,
                     void* stream) {
  TRY(check_device(p));
  if (!b || !x || !(rtol > 0.0) || maxit < 1) return fail(CMG_EINVAL, "bad solve arguments");
  if (p->ghost_local)
    return fail(CMG_EINVAL, "CG needs the symmetric V-cycle: the patch-local ghost coupling is for GMRES and "
                            "the V-cycle iteration");
  auto s = static_cast<hipStream_t>(stream);
  const int L = p->H.cfg.n_levels - 1;
  const int64_t n = p->H.levels[L].n_dofs;
  if (info) *info = cmg_solve_info{0, 0.0, 0.0};
  {
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_fill(n, 0.0, x, s));        // x = 0
    HIP_TRY(cmg::launch_copy(n, b, p->kr, s));      // r = b
  }
  double bb;
  TRY(dot(p, b, b, n, s, &bb));
  const double nb = std::sqrt(bb);
  if (!std::isfinite(nb)) return fail(CMG_EINVAL, "right-hand side is not finite");
  if (nb == 0.0) return CMG_OK;
  TRY(vcycle_current(p, p->kr, p->kz, s));
  {
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_copy(n, p->kz, p->kp, s));  // p = z
  }
  double rz;
  TRY(dot(p, p->kr, p->kz, n, s, &rz));
  for (int it = 1; it <= maxit; ++it) {
    TRY(op_apply<double>(p, L, p->kp, p->kq, s));  // q = A p in FP64
    double pq;
    TRY(dot(p, p->kp, p->kq, n, s, &pq));
    if (!(pq > 0.0) || !std::isfinite(pq)) return fail(CMG_EBREAKDOWN, "CG breakdown: p^T A p <= 0");
    const double alpha = rz / pq;
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_axpy(n, alpha, p->kp, x, s));
      HIP_TRY(cmg::launch_axpy(n, -alpha, p->kq, p->kr, s));
    }
    double rr;
    TRY(dot(p, p->kr, p->kr, n, s, &rr));
    const double rel = std::sqrt(rr) / nb;
    if (info) {
      info->iterations = it;
      info->rel_residual = rel;
      info->n_frac = rel > 0.0 ? it * std::log10(rtol) / std::log10(rel) : it;
    }
    if (rel <= rtol) return CMG_OK;
    TRY(vcycle_current(p, p->kr, p->kz, s));
    double rz_new;
    TRY(dot(p, p->kr, p->kz, n, s, &rz_new));
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_xpay(n, rz_new / rz, p->kz, p->kp, s));
    }
    rz = rz_new;
  }
  return fail(CMG_ENOTCONV, "CG did not converge within maxit");
}

cmg_status cmg_gmres(cmg_problem* p, const double* b, double* x, double rtol, int maxit, int restart,
                     cmg_solve_info* info, void* stream) {
  TRY(check_device(p));
  if (!b || !x || !(rtol > 0.0) || maxit < 1 || restart < 1 || restart >= cmg::kMaxRows)
    return fail(CMG_EINVAL, "bad GMRES arguments (1 <= restart < 64)");
  TRY(ensure_gmres(p, restart));
  auto s = static_cast<hipStream_t>(stream);
  const int L = p->H.cfg.n_levels - 1;
  const int64_t n = p->H.levels[L].n_dofs;
  if (info) *info = cmg_solve_info{0, 0.0, 0.0};
  {
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_fill(n, 0.0, x, s));  // x = 0
  }
  double bb;
  TRY(dot(p, b, b, n, s, &bb));
  const double nb = std::sqrt(bb);
  if (!std::isfinite(nb)) return fail(CMG_EINVAL, "right-hand side is not finite");
  if (nb == 0.0) return CMG_OK;
  double* V = p->gV;
  double* Z = p->gZ;
  double* w = p->gw;
  std::vector<double> H((restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h(restart + 1),
      h2(restart + 1);
  auto Hm = [&](int i, int j) -> double& { return H[i * restart + j]; };
  int it = 0;
  while (it < maxit) {
    // r = b - A x into V_0
    {
      TRY(op_apply<double>(p, L, x, w, s));
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_copy(n, b, V, s));
      HIP_TRY(cmg::launch_axpy(n, -1.0, w, V, s));
    }
    double rr;
    TRY(dot(p, V, V, n, s, &rr));
    const double beta = std::sqrt(rr);
    if (beta <= rtol * nb) return CMG_OK;
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_scale(n, 1.0 / beta, V, V, s));
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jdone = 0;
    bool converged = false;
    for (int j = 0; j < restart; ++j) {
      double* Vj = V + static_cast<int64_t>(j) * n;
      double* Zj = Z + static_cast<int64_t>(j) * n;
      TRY(vcycle_current(p, Vj, Zj, s));      // z_j = B v_j
      TRY(op_apply<double>(p, L, Zj, w, s));  // w = A z_j
      // classical Gram-Schmidt, twice
      cmg::RowCoef c{};
      TRY(rows_dot(p, V, w, n, j + 1, s, h.data()));
      for (int i = 0; i <= j; ++i) c.v[i] = -h[i];
      {
        KTimer t(p, kVector, L, s);
        HIP_TRY(cmg::launch_rows_combine(n, j + 1, c, V, w, s));
      }
      TRY(rows_dot(p, V, w, n, j + 1, s, h2.data()));
      for (int i = 0; i <= j; ++i) {
        c.v[i] = -h2[i];
        h[i] += h2[i];
      }
      {
        KTimer t(p, kVector, L, s);
        HIP_TRY(cmg::launch_rows_combine(n, j + 1, c, V, w, s));
      }
      double ww;
      TRY(dot(p, w, w, n, s, &ww));
      const double hn = std::sqrt(ww);
      if (!std::isfinite(hn)) return fail(CMG_EBREAKDOWN, "GMRES breakdown: non-finite Arnoldi vector");
      if (hn > 0.0) {
        KTimer t(p, kVector, L, s);
        HIP_TRY(cmg::launch_scale(n, 1.0 / hn, w, V + static_cast<int64_t>(j + 1) * n, s));
      }
      for (int i = 0; i <= j; ++i) Hm(i, j) = h[i];
      Hm(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {  // earlier rotations on the new column
        const double t1 = cs[i] * Hm(i, j) + sn[i] * Hm(i + 1, j);
        Hm(i + 1, j) = -sn[i] * Hm(i, j) + cs[i] * Hm(i + 1, j);
        Hm(i, j) = t1;
      }
      const double den = std::hypot(Hm(j, j), Hm(j + 1, j));
      if (!(den > 0.0)) return fail(CMG_EBREAKDOWN, "GMRES breakdown: singular Hessenberg column");
      cs[j] = Hm(j, j) / den;
      sn[j] = Hm(j + 1, j) / den;
      Hm(j, j) = den;
      Hm(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jdone = j + 1;
      const double rel = std::fabs(g[j + 1]) / nb;
      if (info) {
        info->iterations = it;
        info->rel_residual = rel;
        info->n_frac = rel > 0.0 ? it * std::log10(rtol) / std::log10(rel) : it;
      }
      if (rel <= rtol || it >= maxit) {
        converged = rel <= rtol;
        break;
      }
    }
    // x += Z y with H y = g (upper triangular)
    cmg::RowCoef y{};
    for (int i = jdone - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k2 = i + 1; k2 < jdone; ++k2) acc -= Hm(i, k2) * y.v[k2];
      y.v[i] = acc / Hm(i, i);
    }
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_rows_combine(n, jdone, y, Z, x, s));
    }
    if (converged) return CMG_OK;
  }
  return fail(CMG_ENOTCONV, "GMRES did not converge within maxit");
}

cmg_status cmg_vcycle_solve(cmg_problem* p, const double* b, double* x, double rtol, int maxit, cmg_solve_info* info,
                            void* stream) {
  TRY(check_device(p));
  if (!b || !x || !(rtol > 0.0) || maxit < 1) return fail(CMG_EINVAL, "bad V-cycle solver arguments");
  auto s = static_cast<hipStream_t>(stream);
  const int L = p->H.cfg.n_levels - 1;
  const int64_t n = p->H.levels[L].n_dofs;
  if (info) *info = cmg_solve_info{0, 0.0, 0.0};
  {
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_fill(n, 0.0, x, s));    // x = 0
    HIP_TRY(cmg::launch_copy(n, b, p->kr, s));  // r = b
  }
  double bb;
  TRY(dot(p, b, b, n, s, &bb));
  const double nb = std::sqrt(bb);
  if (!std::isfinite(nb)) return fail(CMG_EINVAL, "right-hand side is not finite");
  if (nb == 0.0) return CMG_OK;
  for (int it = 1; it <= maxit; ++it) {
    TRY(vcycle_current(p, p->kr, p->kz, s));  // z = B r
    TRY(op_apply<double>(p, L, p->kz, p->kq, s));
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_axpy(n, 1.0, p->kz, x, s));      // x += z
      HIP_TRY(cmg::launch_axpy(n, -1.0, p->kq, p->kr, s));  // r -= A z (= b - A x)
    }
    double rr;
    TRY(dot(p, p->kr, p->kr, n, s, &rr));
    const double rel = std::sqrt(rr) / nb;
    if (info) {
      info->iterations = it;
      info->rel_residual = rel;
      info->n_frac = rel > 0.0 ? it * std::log10(rtol) / std::log10(rel) : it;
    }
    if (rel <= rtol) return CMG_OK;
    if (!(rel <= 1e3)) return fail(CMG_ENOTCONV, "V-cycle iteration diverges");
  }
  return fail(CMG_ENOTCONV, "V-cycle iteration did not converge within maxit");
}

cmg_status cmg_vcycle_multi(cmg_problem* p, int nrhs, const double* r, double* z, void* stream) {
  TRY(check_device(p));
  if (!r || !z || nrhs < 1 || nrhs > cmg::kMaxCols) return fail(CMG_EINVAL, "bad multi-column V-cycle arguments");
  if (p->ghost_local) return fail(CMG_EINVAL, "multi-column calls run with the exact ghost coupling only");
  TRY(prepare_multi(p));
  return vcycle_multi_current(p, nrhs, r, z, static_cast<hipStream_t>(stream));
}

cmg_status cmg_solve_multi(cmg_problem* p, int nrhs, const double* b, double* x, double rtol, int maxit,
                           cmg_solve_info* info, void* stream) {
  TRY(check_device(p));
  if (!b || !x || !(rtol > 0.0) || maxit < 1 || nrhs < 1 || nrhs > cmg::kMaxCols)
    return fail(CMG_EINVAL, "bad multi-column solve arguments");
  if (p->ghost_local) return fail(CMG_EINVAL, "multi-column calls run with the exact ghost coupling only");
  TRY(prepare_multi(p));
  auto s = static_cast<hipStream_t>(stream);
  const int L = p->H.cfg.n_levels - 1;
  const int64_t n = p->H.levels[L].n_dofs;
  const int64_t nt = n * nrhs;
  if (info)
    for (int c = 0; c < nrhs; ++c) info[c] = cmg_solve_info{0, 0.0, 0.0};
  {
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_fill(nt, 0.0, x, s));       // x = 0
    HIP_TRY(cmg::launch_copy(nt, b, p->mkr, s));    // r = b
  }
  double nb[cmg::kMaxCols], rz[cmg::kMaxCols], tmp[cmg::kMaxCols];
  bool done[cmg::kMaxCols];
  TRY(dot_cols(p, b, b, n, nrhs, s, tmp));
  bool all_done = true;
  for (int c = 0; c < nrhs; ++c) {
    nb[c] = std::sqrt(tmp[c]);
    if (!std::isfinite(nb[c])) return fail(CMG_EINVAL, "right-hand side is not finite");
    done[c] = nb[c] == 0.0;
    all_done = all_done && done[c];
  }
  if (all_done) return CMG_OK;
  TRY(vcycle_multi_current(p, nrhs, p->mkr, p->mkz, s));
  {
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_copy(nt, p->mkz, p->mkp, s));  // p = z
  }
  TRY(dot_cols(p, p->mkr, p->mkz, n, nrhs, s, rz));
  for (int it = 1; it <= maxit; ++it) {
    TRY(op_apply_multi(p, nrhs, p->mkp, p->mkq, s));  // q = A p in FP64
    TRY(dot_cols(p, p->mkp, p->mkq, n, nrhs, s, tmp));
    cmg::ColCoef alpha{}, malpha{};
    for (int c = 0; c < nrhs; ++c) {
      if (done[c]) continue;  // a converged column keeps x and r (alpha = 0)
      if (!(tmp[c] > 0.0) || !std::isfinite(tmp[c])) return fail(CMG_EBREAKDOWN, "CG breakdown: p^T A p <= 0");
      alpha.v[c] = rz[c] / tmp[c];
      malpha.v[c] = -alpha.v[c];
    }
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_axpy_cols(n, alpha, p->mkp, x, nrhs, s));
      HIP_TRY(cmg::launch_axpy_cols(n, malpha, p->mkq, p->mkr, nrhs, s));
    }
    TRY(dot_cols(p, p->mkr, p->mkr, n, nrhs, s, tmp));
    all_done = true;
    for (int c = 0; c < nrhs; ++c) {
      if (done[c]) continue;
      const double rel = std::sqrt(tmp[c]) / nb[c];
      if (info) {
        info[c].iterations = it;
        info[c].rel_residual = rel;
        info[c].n_frac = rel > 0.0 ? it * std::log10(rtol) / std::log10(rel) : it;
      }
      done[c] = rel <= rtol;
      all_done = all_done && done[c];
    }
    if (all_done) return CMG_OK;
    TRY(vcycle_multi_current(p, nrhs, p->mkr, p->mkz, s));
    TRY(dot_cols(p, p->mkr, p->mkz, n, nrhs, s, tmp));
    cmg::ColCoef beta{};
    for (int c = 0; c < nrhs; ++c) {
      beta.v[c] = done[c] ? 0.0 : tmp[c] / rz[c];
      rz[c] = tmp[c];
    }
    {
      KTimer t(p, kVector, L, s);
      HIP_TRY(cmg::launch_xpay_cols(n, beta, p->mkz, p->mkp, nrhs, s));
    }
  }
  return fail(CMG_ENOTCONV, "CG did not converge within maxit for every column");
}

cmg_status cmg_group_create(cmg_problem* const* members, int n, cmg_group** out) {
  if (!out || !members || n < 1 || n > kMaxGroup) return fail(CMG_EINVAL, "bad group arguments (1..8 members)");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    TRY(check_device(members[i]));
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return fail(CMG_EINVAL, "a problem appears twice in the group");
  }
  const cmg_problem* p0 = members[0];
  for (int i = 1; i < n; ++i) {
    const cmg_problem* p = members[i];
    const cmg::Config &a = p0->H.cfg, &b = p->H.cfg;
    if (a.dim != b.dim || a.k != b.k || a.n_levels != b.n_levels || a.coarse_cells != b.coarse_cells ||
        a.lo != b.lo || a.hi != b.hi || p->fp32 != p0->fp32 || p->device != p0->device)
      return fail(CMG_EINVAL, "group members differ in dimension, degree, levels, coarse mesh, box, precision or "
                              "device");
  }
  for (int i = 0; i < n; ++i) {
    if (members[i]->ghost_local) return fail(CMG_EINVAL, "group members run with the exact ghost coupling only");
    TRY(prepare_multi(members[i]));
  }
  auto* g = new cmg_group();
  g->m.assign(members, members + n);
  g->fp32 = p0->fp32;
  for (int i = 0; i < n; ++i) g->use_graph = g->use_graph && members[i]->use_graphs;
  const cmg_status st = g->fp32 ? group_plan<float>(g) : group_plan<double>(g);
  if (st != CMG_OK) {
    group_release(g);
    delete g;
    return st;
  }
  *out = g;
  return CMG_OK;
}

void cmg_group_destroy(cmg_group* g) {
  if (!g) return;
  group_release(g);
  delete g;
}

cmg_status cmg_group_vcycle(cmg_group* g, const double* const* r, double* const* z, void* stream) {
  if (!g || !r || !z) return fail(CMG_EINVAL, "null argument");
  for (size_t i = 0; i < g->m.size(); ++i)
    if (!r[i] || !z[i]) return fail(CMG_EINVAL, "null member vector");
  return group_vcycle(g, r, z, static_cast<hipStream_t>(stream));
}

cmg_status cmg_group_solve(cmg_group* g, const double* const* b, double* const* x, double rtol, int maxit,
                           cmg_solve_info* info, cmg_status* status, void* stream) {
  if (!g || !b || !x || !(rtol > 0.0) || maxit < 1) return fail(CMG_EINVAL, "bad group solve arguments");
  const int G = static_cast<int>(g->m.size());
  for (int i = 0; i < G; ++i)
    if (!b[i] || !x[i]) return fail(CMG_EINVAL, "null member vector");
  auto s = static_cast<hipStream_t>(stream);
  // every member runs the recurrence of cmg_solve_multi with one column, on
  // its own multi-column Krylov vectors; a member that converged or failed is
  // frozen while the others continue
  std::vector<int64_t> n(G);
  std::vector<double> nb(G), rz(G);
  std::vector<cmg_status> st(G, CMG_OK);
  std::vector<bool> done(G, false);
  std::vector<const double*> R(G);
  std::vector<double*> Zw(G);
  std::string msg;
  auto stop = [&](int i, cmg_status code, const char* what) {
    st[i] = code;
    done[i] = true;
    if (msg.empty()) msg = std::string(what) + " (member " + std::to_string(i) + ")";
  };
  for (int i = 0; i < G; ++i) {
    cmg_problem* p = g->m[i];
    const int L = p->H.cfg.n_levels - 1;
    n[i] = p->H.levels[L].n_dofs;
    if (info) info[i] = cmg_solve_info{0, 0.0, 0.0};
    R[i] = p->mkr;
    Zw[i] = p->mkz;
    KTimer t(p, kVector, L, s);
    HIP_TRY(cmg::launch_fill(n[i], 0.0, x[i], s));     // x = 0
    HIP_TRY(cmg::launch_copy(n[i], b[i], p->mkr, s));  // r = b
  }
  // the dot products of all members are queued together and summed after one
  // wait (the same partial sums and the same host sums as dot_cols)
  auto dots = [&](const std::vector<int>& who, auto&& vecs, std::vector<double>& out) -> cmg_status {
    for (int i : who) {
      const std::pair<const double*, const double*> v = vecs(i);
      TRY(dot_cols_start(g->m[i], v.first, v.second, n[i], 1, s));
    }
    if (!who.empty()) TRY(wait_stream(g->m[who.front()], s));
    for (int i : who) dot_cols_sum(g->m[i], 1, &out[i]);
    return CMG_OK;
  };
  auto active = [&]() {
    std::vector<int> a;
    for (int i = 0; i < G; ++i)
      if (!done[i]) a.push_back(i);
    return a;
  };
  std::vector<double> tmp(G, 0.0);
  std::vector<int> all(G);
  for (int i = 0; i < G; ++i) all[i] = i;
  TRY(dots(all, [&](int i) { return std::make_pair(b[i], b[i]); }, tmp));
  bool all_done = true;
  for (int i = 0; i < G; ++i) {
    nb[i] = std::sqrt(tmp[i]);
    if (!std::isfinite(nb[i])) stop(i, CMG_EINVAL, "right-hand side is not finite");
    else done[i] = nb[i] == 0.0;
    all_done = all_done && done[i];
  }
  if (!all_done) {
    TRY(group_vcycle(g, R.data(), Zw.data(), s));
    const std::vector<int> a = active();
    for (int i : a) {
      cmg_problem* p = g->m[i];
      KTimer t(p, kVector, p->H.cfg.n_levels - 1, s);
      HIP_TRY(cmg::launch_copy(n[i], p->mkz, p->mkp, s));  // p = z
    }
    TRY(dots(a, [&](int i) { return std::pair<const double*, const double*>(g->m[i]->mkr, g->m[i]->mkz); },
             rz));
  }
  for (int it = 1; it <= maxit && !all_done; ++it) {
    std::vector<int> a = active();
    for (int i : a) TRY(op_apply_multi(g->m[i], 1, g->m[i]->mkp, g->m[i]->mkq, s));  // q = A p in FP64
    TRY(dots(a, [&](int i) { return std::pair<const double*, const double*>(g->m[i]->mkp, g->m[i]->mkq); },
             tmp));
    std::vector<int> upd;
    for (int i : a) {
      if (!(tmp[i] > 0.0) || !std::isfinite(tmp[i])) {
        stop(i, CMG_EBREAKDOWN, "CG breakdown: p^T A p <= 0");
        continue;
      }
      cmg_problem* p = g->m[i];
      cmg::ColCoef alpha{}, malpha{};
      alpha.v[0] = rz[i] / tmp[i];
      malpha.v[0] = -alpha.v[0];
      KTimer t(p, kVector, p->H.cfg.n_levels - 1, s);
      HIP_TRY(cmg::launch_axpy_cols(n[i], alpha, p->mkp, x[i], 1, s));
      HIP_TRY(cmg::launch_axpy_cols(n[i], malpha, p->mkq, p->mkr, 1, s));
      upd.push_back(i);
    }
    TRY(dots(upd, [&](int i) { return std::pair<const double*, const double*>(g->m[i]->mkr, g->m[i]->mkr); },
             tmp));
    for (int i : upd) {
      const double rel = std::sqrt(tmp[i]) / nb[i];
      if (info) {
        info[i].iterations = it;
        info[i].rel_residual = rel;
        info[i].n_frac = rel > 0.0 ? it * std::log10(rtol) / std::log10(rel) : it;
      }
      done[i] = rel <= rtol;
    }
    a = active();
    if (a.empty()) break;
    TRY(group_vcycle(g, R.data(), Zw.data(), s));
    TRY(dots(a, [&](int i) { return std::pair<const double*, const double*>(g->m[i]->mkr, g->m[i]->mkz); },
             tmp));
    for (int i : a) {
      cmg_problem* p = g->m[i];
      cmg::ColCoef beta{};
      beta.v[0] = tmp[i] / rz[i];
      rz[i] = tmp[i];
      KTimer t(p, kVector, p->H.cfg.n_levels - 1, s);
      HIP_TRY(cmg::launch_xpay_cols(n[i], beta, p->mkz, p->mkp, 1, s));
    }
  }
  for (int i = 0; i < G; ++i)
    if (!done[i]) stop(i, CMG_ENOTCONV, "CG did not converge within maxit");
  if (status)
    for (int i = 0; i < G; ++i) status[i] = st[i];
  for (int i = 0; i < G; ++i)
    if (st[i] != CMG_OK) return fail(st[i], msg);
  return CMG_OK;
}

cmg_status cmg_timing(cmg_problem* p, unsigned kind_mask) {
  TRY(check_device(p));
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
  HIP_TRY(hipDeviceSynchronize());
  const int lv = static_cast<int>((kind_mask >> 16) & 0xffu) - 1;
  if (lv >= static_cast<int>(p->lv.size())) return fail(CMG_EINVAL, "timing level out of range");
  p->timing_mask = kind_mask & 0xffffu;
  p->timing_level = lv;
  p->recs.clear();
  p->pool_used = 0;
  drop_graphs(p);  // recaptured with (or without) the timed launches as pieces of their own
  // create the events now rather than inside the timed launches
  while (p->timing_mask && p->pool.size() < 8192) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    p->pool.push_back(e);
  }
  return CMG_OK;
}

cmg_status cmg_timing_read(cmg_problem* p, int kind, int level, int64_t* launches, double* total_ms) {
  TRY(check_device(p));
  if (!launches || !total_ms) return fail(CMG_EINVAL, "null output");
  *launches = 0;
  *total_ms = 0.0;
  for (const auto& r : p->recs) {
    if (r.kind != kind || (level >= 0 && r.level != level)) continue;
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    *launches += r.n;
    *total_ms += ms;
  }
  return CMG_OK;
}

cmg_status cmg_rhs_manufactured(const cmg_problem* p, double* b_host) {
  if (!p || !b_host) return fail(CMG_EINVAL, "null argument");
  std::vector<double> b;
  cmg::manufactured_rhs(p->H, b);
  std::memcpy(b_host, b.data(), b.size() * sizeof(double));
  return CMG_OK;
}

cmg_status cmg_rhs_fourier(const cmg_problem* p, int n_modes, const int* kappa, const double* amp,
                           const double* phase, double* b_host) {
  if (!p || !b_host || n_modes < 0 || (n_modes > 0 && (!kappa || !amp || !phase)))
    return fail(CMG_EINVAL, "bad Fourier right-hand side");
  std::vector<double> b;
  cmg::fourier_rhs(p->H, n_modes, kappa, amp, phase, b);
  std::memcpy(b_host, b.data(), b.size() * sizeof(double));
  return CMG_OK;
}

cmg_status cmg_export(const cmg_problem* p, int level, int what, void* buf, size_t bytes, size_t* needed) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (level < 0 || level >= p->H.cfg.n_levels) return fail(CMG_EINVAL, "level out of range");
  const cmg::HostLevel& h = p->H.levels[level];
  std::vector<int64_t> counts;
  std::vector<double> quad;
  const void* src = nullptr;
  size_t sz = 0;
  if (what == 0) {
    int64_t active = 0, ghost = 0, sumsq = 0;
    for (int64_t c = 0; c < h.n_cells; ++c) {
      active += (h.cell_flags[c] & cmg::kActive) != 0;
      for (int dir = 0; dir < p->H.cfg.dim; ++dir) ghost += (h.ghost_mask[c] >> (2 * dir + 1)) & 1;
    }
    for (int c = 0; c < 8; ++c)
      for (size_t i = 0; i + 1 < h.cut[c].off.size(); ++i) {
        const int64_t nj = h.cut[c].off[i + 1] - h.cut[c].off[i];
        sumsq += nj * nj;
      }
    counts = {h.n_dofs, active, h.n_cut, h.n_int_patches, h.n_cut_patches, sumsq, ghost, h.nn};
    src = counts.data();
    sz = counts.size() * sizeof(int64_t);
  } else if (what == 1) {
    src = h.dof_node.data();
    sz = h.dof_node.size() * sizeof(int32_t);
  } else if (what == 2) {
    src = h.cell_flags.data();
    sz = h.cell_flags.size();
  } else if (what == 3) {
    src = h.cut_mats.data();
    sz = h.cut_mats.size() * sizeof(double);
  } else if (what == 5) {
    // the cut-cell rule of the element matrices (columns), per cut cell in cut-id order
    const cmg::Config& cfg = p->H.cfg;
    const int d = cfg.dim;
    for (int64_t c = 0; c < h.n_cells; ++c) {
      if (h.cut_id[c] < 0) continue;
      double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      for (int j = 0, r = static_cast<int>(c); j < d; ++j) {
        lo[j] = cfg.lo + (r % h.N) * h.h;
        hi[j] = lo[j] + h.h;
        r /= h.N;
      }
      std::vector<cmg::Column> cols;
      cmg::cut_columns_union(d, cfg.shapes, lo, hi, cfg.quad_n, cfg.k + 1, cfg.quad_beta, cfg.union_depth, cols);
      quad.push_back(static_cast<double>(cols.size()));
      for (const cmg::Column& col : cols) {
        quad.push_back(col.e);
        for (int j = 0; j < d; ++j) quad.push_back(col.x[j]);
        quad.push_back(col.w);
        quad.push_back(col.t0);
        quad.push_back(col.t1);
        quad.push_back(col.surf ? 1.0 : 0.0);
        quad.push_back(col.ts);
        quad.push_back(col.sw);
        for (int j = 0; j < d; ++j) quad.push_back(col.nrm[j]);
      }
    }
    src = quad.data();
    sz = quad.size() * sizeof(double);
  } else if (what == 4) {
    if (level != 0) return fail(CMG_EINVAL, "the coarse inverse lives on level 0");
    src = p->H.coarse_inv.data();
    sz = p->H.coarse_inv.size() * sizeof(double);
  } else if (what >= 16 && what < 24) {
    src = h.int_vertex[what - 16].data();
    sz = h.int_vertex[what - 16].size() * sizeof(int32_t);
  } else if (what >= 24 && what < 32) {
    src = h.cut[what - 24].off.data();
    sz = h.cut[what - 24].off.size() * sizeof(int32_t);
  } else if (what >= 32 && what < 40) {
    src = h.cut[what - 32].nodes.data();
    sz = h.cut[what - 32].nodes.size() * sizeof(int32_t);
  } else if (what >= 40 && what < 48) {
    src = h.cut[what - 40].inv.data();
    sz = h.cut[what - 40].inv.size() * sizeof(double);
  } else if (what >= 48 && what < 56) {
    src = h.cut[what - 48].vertex.data();
    sz = h.cut[what - 48].vertex.size() * sizeof(int32_t);
  } else if (what >= 56 && what < 64) {
    src = h.cut[what - 56].nxt.data();
    sz = h.cut[what - 56].nxt.size();
  } else if (what == 64) {
    src = h.cut_region.data();
    sz = h.cut_region.size() * sizeof(int32_t);
  } else {
    return fail(CMG_EINVAL, "unknown export kind");
  }
  if (needed) *needed = sz;
  if (!buf) return CMG_OK;
  if (bytes < sz) return fail(CMG_EINVAL, "export buffer too small");
  std::memcpy(buf, src, sz);
  return CMG_OK;
}

}  // extern "C"
