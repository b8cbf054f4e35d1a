// C ABI of the CutFEM vertex-patch multigrid: device upload of the hierarchy,
// V-cycle orchestration (paper Section 2.2) and preconditioned CG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
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

#define HIP_TRY(...)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (__VA_ARGS__);                                                            \
    if (e_ != hipSuccess) return fail(CMG_EHIP, std::string(#__VA_ARGS__ ": ") + hipGetErrorString(e_)); \
  } while (0)

struct DevLevel {
  cmg::KLevel kl{};
  std::vector<void*> owned;
  double* x = nullptr;   // lattice work vectors
  double* b = nullptr;
  double* r = nullptr;
  double* dbuf = nullptr;
  int32_t* int_verts[8] = {};
  int n_int[8] = {};
  cmg::CutGroupDev cut[8] = {};
};

}  // namespace

struct cmg_problem {
  cmg::Hierarchy H;
  std::vector<DevLevel> lv;
  double* coarse_inv = nullptr;
  std::vector<void*> owned;
  // Krylov vectors (compact, finest level)
  double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr, *part = nullptr;
  double* part_host = nullptr;
  int nblk = 0;
  int device = 0;
  // kernel timing: launches of the kinds in timing_mask are bracketed by events
  unsigned timing_mask = 0;
  struct Rec { int kind, level; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

namespace {

template <typename T>
cmg_status upload(cmg_problem* P, std::vector<void*>& owned, const std::vector<T>& host, T** dptr) {
  *dptr = nullptr;
  if (host.empty()) return CMG_OK;
  void* p = nullptr;
  if (hipMalloc(&p, host.size() * sizeof(T)) != hipSuccess) return fail(CMG_ENOMEM, "device allocation failed");
  owned.push_back(p);
  HIP_TRY(hipMemcpy(p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
  *dptr = static_cast<T*>(p);
  return CMG_OK;
}

cmg_status alloc_zero(std::vector<void*>& owned, size_t bytes, void** dptr) {
  *dptr = nullptr;
  if (bytes == 0) return CMG_OK;
  if (hipMalloc(dptr, bytes) != hipSuccess) return fail(CMG_ENOMEM, "device allocation failed");
  owned.push_back(*dptr);
  HIP_TRY(hipMemset(*dptr, 0, bytes));
  return CMG_OK;
}

#define TRY(expr)                       \
  do {                                  \
    cmg_status s_ = (expr);             \
    if (s_ != CMG_OK) return s_;        \
  } while (0)

cmg_status upload_all(cmg_problem* P) {
  const cmg::Config& cfg = P->H.cfg;
  const int L = cfg.n_levels;
  P->lv.resize(L);
  for (int l = 0; l < L; ++l) {
    const cmg::HostLevel& h = P->H.levels[l];
    DevLevel& d = P->lv[l];
    d.kl.N = h.N;
    d.kl.nn = h.nn;
    d.kl.n_dofs = h.n_dofs;
    uint8_t* flags;
    int32_t* cut_id;
    uint8_t* ghost;
    double* cm;
    int32_t* dn;
    double* tab;
    TRY(upload(P, d.owned, h.cell_flags, &flags));
    TRY(upload(P, d.owned, h.cut_id, &cut_id));
    TRY(upload(P, d.owned, h.ghost_mask, &ghost));
    TRY(upload(P, d.owned, h.cut_mats, &cm));
    TRY(upload(P, d.owned, h.dof_node, &dn));
    const cmg::LevelTables& t = P->H.tables[l];
    std::vector<double> packed;
    for (const auto* v : {&t.kcell, &t.mhat, &t.d0, &t.d1, &t.gcoef, &t.fd_s, &t.fd_dinv, &t.p1d})
      packed.insert(packed.end(), v->begin(), v->end());
    if (static_cast<int>(packed.size()) != cmg::tables_size(cfg.dim, cfg.k))
      return fail(CMG_EINVAL, "internal: table layout mismatch");
    TRY(upload(P, d.owned, packed, &tab));
    d.kl.flags = flags;
    d.kl.cut_id = cut_id;
    d.kl.ghost = ghost;
    d.kl.cut_mats = cm;
    d.kl.dof_node = dn;
    d.kl.tables = tab;
    const size_t lat_bytes = static_cast<size_t>(h.n_nodes) * sizeof(double);
    TRY(alloc_zero(d.owned, lat_bytes, reinterpret_cast<void**>(&d.x)));
    TRY(alloc_zero(d.owned, lat_bytes, reinterpret_cast<void**>(&d.b)));
    TRY(alloc_zero(d.owned, lat_bytes, reinterpret_cast<void**>(&d.r)));
    int64_t maxn = 0;
    for (int c = 0; c < 8; ++c) {
      TRY(upload(P, d.owned, h.int_vertex[c], &d.int_verts[c]));
      d.n_int[c] = static_cast<int>(h.int_vertex[c].size());
      const cmg::CutPatchGroup& g = h.cut[c];
      cmg::CutGroupDev& G = d.cut[c];
      G.n_patch = static_cast<int>(g.vertex.size());
      G.n_nodes = static_cast<int64_t>(g.nodes.size());
      if (G.n_patch == 0) continue;
      int32_t* off;
      int64_t* ioff;
      int32_t* nodes;
      double* inv;
      TRY(upload(P, d.owned, g.off, &off));
      TRY(upload(P, d.owned, g.inv_off, &ioff));
      TRY(upload(P, d.owned, g.nodes, &nodes));
      TRY(upload(P, d.owned, g.inv, &inv));
      G.off = off;
      G.inv_off = ioff;
      G.nodes = nodes;
      G.inv = inv;
      maxn = std::max(maxn, G.n_nodes);
    }
    TRY(alloc_zero(d.owned, static_cast<size_t>(maxn) * sizeof(double), reinterpret_cast<void**>(&d.dbuf)));
  }
  TRY(upload(P, P->owned, P->H.coarse_inv, &P->coarse_inv));
  const int64_t n = P->H.levels.back().n_dofs;
  for (double** v : {&P->kr, &P->kz, &P->kp, &P->kq})
    TRY(alloc_zero(P->owned, n * sizeof(double), reinterpret_cast<void**>(v)));
  P->nblk = static_cast<int>(std::min<int64_t>(1024, (n + 255) / 256));
  TRY(alloc_zero(P->owned, P->nblk * sizeof(double), reinterpret_cast<void**>(&P->part)));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->part_host), P->nblk * sizeof(double), hipHostMallocDefault));
  return CMG_OK;
}

cmg_status check_device(const cmg_problem* p) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (p->lv.empty()) return fail(CMG_EINVAL, "problem was set up on the host only");
  return CMG_OK;
}

cmg_status check_level(const cmg_problem* p, int level, bool need_fine) {
  if (!p) return fail(CMG_EINVAL, "null problem");
  if (level < (need_fine ? 1 : 0) || level >= p->H.cfg.n_levels) return fail(CMG_EINVAL, "level out of range");
  return CMG_OK;
}

// Brackets one kernel launch with HIP events when its kind is being timed.
struct KTimer {
  cmg_problem* P;
  int kind, level;
  hipStream_t s;
  hipEvent_t b = nullptr;
  KTimer(cmg_problem* P_, int kind_, int level_, hipStream_t s_) : P(P_), kind(kind_), level(level_), s(s_) {
    if (!(P->timing_mask & (1u << kind))) return;
    if (P->pool_used + 2 > P->pool.size()) {
      for (int i = 0; i < 1024; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        P->pool.push_back(e);
      }
    }
    hipEvent_t a = P->pool[P->pool_used++];
    b = P->pool[P->pool_used++];
    (void)hipEventRecord(a, s);
    P->recs.push_back({kind, level, a, b});
  }
  ~KTimer() {
    if (b) (void)hipEventRecord(b, s);
  }
};

enum KernelKind { kApply = 0, kInterior = 1, kCutSolve = 2, kCutUpdate = 3, kProlong = 4, kRestrict = 5,
                  kCoarse = 6, kLayout = 7, kVector = 8 };

// ---- device-side building blocks on the internal lattice vectors ------------

cmg_status colour_step(cmg_problem* P, int l, bool interior, int colour, hipStream_t s) {
  const int d = P->H.cfg.dim, k = P->H.cfg.k;
  DevLevel& D = P->lv[l];
  if (interior) {
    if (D.n_int[colour] == 0) return CMG_OK;
    KTimer t(P, kInterior, l, s);
    HIP_TRY(cmg::launch_interior_step<double>(d, k, D.kl, D.int_verts[colour], D.n_int[colour], D.x, D.b, s));
  } else {
    if (D.cut[colour].n_patch == 0) return CMG_OK;
    {
      KTimer t(P, kCutSolve, l, s);
      HIP_TRY(cmg::launch_cut_solve<double>(d, k, D.kl, D.cut[colour], D.x, D.b, D.dbuf, s));
    }
    KTimer t(P, kCutUpdate, l, s);
    HIP_TRY(cmg::launch_cut_update<double>(D.cut[colour], D.dbuf, D.x, s));
  }
  return CMG_OK;
}

cmg_status smooth(cmg_problem* P, int l, bool post, hipStream_t s) {
  const int C = 1 << P->H.cfg.dim;
  std::vector<std::pair<bool, int>> seq;
  for (int c = 0; c < C; ++c) seq.push_back({true, c});
  for (int r = 0; r < P->H.cfg.n_c; ++r)
    for (int c = 0; c < C; ++c) seq.push_back({false, c});
  if (post) std::reverse(seq.begin(), seq.end());
  for (auto [interior, c] : seq) TRY(colour_step(P, l, interior, c, s));
  return CMG_OK;
}

cmg_status coarse(cmg_problem* P, hipStream_t s) {
  DevLevel& D = P->lv[0];
  KTimer t(P, kCoarse, 0, s);
  HIP_TRY(cmg::launch_coarse<double>(P->coarse_inv, D.kl.dof_node, static_cast<int>(P->H.n_coarse), D.b, D.x, s));
  return CMG_OK;
}

// V-cycle on the lattice vectors: lv[L].x = B lv[L].b.
cmg_status vcycle_lattice(cmg_problem* P, hipStream_t s) {
  const int d = P->H.cfg.dim, k = P->H.cfg.k;
  const int L = P->H.cfg.n_levels - 1;
  for (int l = L; l >= 1; --l) {
    DevLevel& D = P->lv[l];
    {
      KTimer t(P, kLayout, l, s);
      HIP_TRY(cmg::launch_zero_active<double>(D.kl.dof_node, D.kl.n_dofs, D.x, s));
    }
    TRY(smooth(P, l, false, s));
    {
      KTimer t(P, kApply, l, s);
      HIP_TRY(cmg::launch_apply<double>(d, k, D.kl, D.x, D.b, D.r, s));
    }
    KTimer t(P, kRestrict, l, s);
    HIP_TRY(cmg::launch_restrict<double>(d, k, P->lv[l - 1].kl, D.kl, D.r, P->lv[l - 1].b, s));
  }
  TRY(coarse(P, s));
  for (int l = 1; l <= L; ++l) {
    DevLevel& D = P->lv[l];
    {
      KTimer t(P, kProlong, l, s);
      HIP_TRY(cmg::launch_prolong_add<double>(d, k, P->lv[l - 1].kl, D.kl, P->lv[l - 1].x, D.x, s));
    }
    TRY(smooth(P, l, true, s));
  }
  return CMG_OK;
}

cmg_status scatter(cmg_problem* P, int l, const double* src, double* lat, hipStream_t s) {
  KTimer t(P, kLayout, l, s);
  HIP_TRY(cmg::launch_scatter<double, double>(P->lv[l].kl.dof_node, P->lv[l].kl.n_dofs, src, lat, s));
  return CMG_OK;
}

cmg_status gather(cmg_problem* P, int l, const double* lat, double* dst, hipStream_t s) {
  KTimer t(P, kLayout, l, s);
  HIP_TRY(cmg::launch_gather<double, double>(P->lv[l].kl.dof_node, P->lv[l].kl.n_dofs, lat, dst, s));
  return CMG_OK;
}

cmg_status dot(cmg_problem* P, const double* x, const double* y, int64_t n, hipStream_t s, double* out) {
  {
    KTimer t(P, kVector, P->H.cfg.n_levels - 1, s);
    HIP_TRY(cmg::launch_dot_partial(x, y, n, P->part, P->nblk, s));
  }
  HIP_TRY(hipMemcpyAsync(P->part_host, P->part, P->nblk * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int i = 0; i < P->nblk; ++i) acc += P->part_host[i];
  *out = acc;
  return CMG_OK;
}

}  // namespace

extern "C" {

const char* cmg_last_error(void) { return g_last_error.c_str(); }

static cmg_status setup_impl(const cmg_levelset* ls, const cmg_params* prm, cmg_problem** out, bool device) {
  g_last_error.clear();
  if (!ls || !prm || !out) return fail(CMG_EINVAL, "null argument");
  *out = nullptr;
  if (ls->dim < 2 || ls->dim > 3 || ls->n_shapes < 1 || !ls->centers || !ls->semi || !(ls->box_hi > ls->box_lo))
    return fail(CMG_EINVAL, "bad level set description");
  if (prm->k < 1 || prm->k > 3 || prm->n_levels < 1 || prm->n_levels > 12 || prm->coarse_cells < 1 ||
      prm->n_c < 0 || prm->quad_n < 2 || prm->quad_n > 64 || prm->ghost_exp_mode < 0 || prm->ghost_exp_mode > 1)
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
  if (cfg.shapes.size() != 1) return fail(CMG_EINVAL, "cut-cell quadrature supports exactly one shape");
  cfg.gamma_D = prm->gamma_D;
  cfg.gamma_g = prm->gamma_g;
  cfg.ghost_exp_mode = prm->ghost_exp_mode;
  cfg.n_c = prm->n_c;
  cfg.quad_n = prm->quad_n;
  auto* P = new cmg_problem();
  std::string err = cmg::build_hierarchy(cfg, P->H);
  if (!err.empty()) {
    delete P;
    cmg_status st = CMG_EINVAL;
    if (err.rfind("EGEOM", 0) == 0) st = CMG_EGEOM;
    if (err.rfind("ENOTSPD", 0) == 0) st = CMG_ENOTSPD;
    return fail(st, err);
  }
  if (!device) {
    *out = P;
    return CMG_OK;
  }
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return fail(CMG_EHIP, "no HIP device");
  }
  cmg_status st = upload_all(P);
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
  for (auto& d : p->lv)
    for (void* v : d.owned) (void)hipFree(v);
  for (void* v : p->owned) (void)hipFree(v);
  if (p->part_host) (void)hipHostFree(p->part_host);
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  delete p;
}

cmg_status cmg_ndofs(const cmg_problem* p, int level, int64_t* n) {
  TRY(check_level(p, level, false));
  if (!n) return fail(CMG_EINVAL, "null output");
  *n = p->H.levels[level].n_dofs;
  return CMG_OK;
}

cmg_status cmg_apply(cmg_problem* p, int level, const double* x, double* y, void* stream) {
  TRY(check_device(p));
  TRY(check_level(p, level, false));
  if (!x || !y) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  DevLevel& D = p->lv[level];
  TRY(scatter(p, level, x, D.x, s));
  HIP_TRY(cmg::launch_apply<double>(p->H.cfg.dim, p->H.cfg.k, D.kl, D.x, nullptr, D.r, s));
  return gather(p, level, D.r, y, s);
}

cmg_status cmg_colour_step(cmg_problem* p, int level, int interior, int colour, double* x, const double* b,
                           void* stream) {
  TRY(check_device(p));
  TRY(check_level(p, level, true));
  if (colour < 0 || colour >= (1 << p->H.cfg.dim)) return fail(CMG_EINVAL, "colour out of range");
  if (!x || !b) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  DevLevel& D = p->lv[level];
  TRY(scatter(p, level, x, D.x, s));
  TRY(scatter(p, level, b, D.b, s));
  TRY(colour_step(p, level, interior != 0, colour, s));
  return gather(p, level, D.x, x, s);
}

cmg_status cmg_smooth(cmg_problem* p, int level, int post, double* x, const double* b, void* stream) {
  TRY(check_device(p));
  TRY(check_level(p, level, true));
  if (!x || !b) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  DevLevel& D = p->lv[level];
  TRY(scatter(p, level, x, D.x, s));
  TRY(scatter(p, level, b, D.b, s));
  TRY(smooth(p, level, post != 0, s));
  return gather(p, level, D.x, x, s);
}

cmg_status cmg_transfer(cmg_problem* p, int level, int dir, const double* x, double* y, void* stream) {
  TRY(check_device(p));
  TRY(check_level(p, level, true));
  if (!x || !y || (dir != 0 && dir != 1)) return fail(CMG_EINVAL, "bad transfer arguments");
  auto s = static_cast<hipStream_t>(stream);
  const int d = p->H.cfg.dim, k = p->H.cfg.k;
  DevLevel& F = p->lv[level];
  DevLevel& C = p->lv[level - 1];
  if (dir == 0) {
    TRY(scatter(p, level - 1, x, C.x, s));
    HIP_TRY(cmg::launch_zero_active<double>(F.kl.dof_node, F.kl.n_dofs, F.x, s));
    HIP_TRY(cmg::launch_prolong_add<double>(d, k, C.kl, F.kl, C.x, F.x, s));
    return gather(p, level, F.x, y, s);
  }
  TRY(scatter(p, level, x, F.r, s));
  HIP_TRY(cmg::launch_restrict<double>(d, k, C.kl, F.kl, F.r, C.b, s));
  return gather(p, level - 1, C.b, y, s);
}

cmg_status cmg_coarse_solve(cmg_problem* p, const double* b, double* x, void* stream) {
  TRY(check_device(p));
  TRY(check_level(p, 0, false));
  if (!x || !b) return fail(CMG_EINVAL, "null vector");
  auto s = static_cast<hipStream_t>(stream);
  TRY(scatter(p, 0, b, p->lv[0].b, s));
  TRY(coarse(p, s));
  return gather(p, 0, p->lv[0].x, x, s);
}

cmg_status cmg_vcycle(cmg_problem* p, const double* r, double* z, void* stream) {
  TRY(check_device(p));
  if (!r || !z) return fail(CMG_EINVAL, "null argument");
  auto s = static_cast<hipStream_t>(stream);
  const int L = p->H.cfg.n_levels - 1;
  TRY(scatter(p, L, r, p->lv[L].b, s));
  TRY(vcycle_lattice(p, s));
  return gather(p, L, p->lv[L].x, z, s);
}

cmg_status cmg_solve(cmg_problem* p, const double* b, double* x, double rtol, int maxit, cmg_solve_info* info,
                     void* stream) {
  TRY(check_device(p));
  if (!b || !x || !(rtol > 0.0) || maxit < 1) return fail(CMG_EINVAL, "bad solve arguments");
  auto s = static_cast<hipStream_t>(stream);
  const int L = p->H.cfg.n_levels - 1;
  const int64_t n = p->H.levels[L].n_dofs;
  const int d = p->H.cfg.dim, k = p->H.cfg.k;
  DevLevel& D = p->lv[L];
  HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), s));
  HIP_TRY(hipMemcpyAsync(p->kr, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double bb;
  TRY(dot(p, b, b, n, s, &bb));
  const double nb = std::sqrt(bb);
  if (info) *info = cmg_solve_info{0, 0.0, 0.0};
  if (nb == 0.0) return CMG_OK;
  TRY(cmg_vcycle(p, p->kr, p->kz, s));
  HIP_TRY(hipMemcpyAsync(p->kp, p->kz, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double rz;
  TRY(dot(p, p->kr, p->kz, n, s, &rz));
  double rel = 1.0;
  for (int it = 1; it <= maxit; ++it) {
    TRY(scatter(p, L, p->kp, D.x, s));
    {
      KTimer t(p, kApply, L, s);
      HIP_TRY(cmg::launch_apply<double>(d, k, D.kl, D.x, nullptr, D.r, s));
    }
    TRY(gather(p, L, D.r, p->kq, s));
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
    rel = std::sqrt(rr) / nb;
    if (info) {
      info->iterations = it;
      info->rel_residual = rel;
      info->n_frac = rel > 0.0 ? it * std::log10(rtol) / std::log10(rel) : it;
    }
    if (rel <= rtol) return CMG_OK;
    TRY(cmg_vcycle(p, p->kr, p->kz, s));
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

cmg_status cmg_timing(cmg_problem* p, unsigned kind_mask) {
  TRY(check_device(p));
  HIP_TRY(hipDeviceSynchronize());
  p->timing_mask = kind_mask;
  p->recs.clear();
  p->pool_used = 0;
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
    *launches += 1;
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

cmg_status cmg_export(const cmg_problem* p, int level, int what, void* buf, size_t bytes, size_t* needed) {
  TRY(check_level(p, level, false));
  const cmg::HostLevel& h = p->H.levels[level];
  std::vector<int64_t> counts;
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
