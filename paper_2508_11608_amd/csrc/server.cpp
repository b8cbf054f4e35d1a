// Continuous-batching solve server on one GPU.
//
// Requests (a level-set domain, discretisation parameters, a right-hand side and
// a tolerance) are queued in arrival order.  Every slot is a worker thread with
// its own HIP stream (default priority).  A free slot takes the oldest request
// and up to kMaxCols - 1 further queued requests with the same geometry,
// parameters, tolerance and iteration limit (a batch), looks for a resident
// hierarchy of that geometry, otherwise reserves its exact device footprint
// (cmg_footprint: counts only, before any quadrature or factorisation) in the
// HBM budget, evicting least-recently used idle hierarchies or waiting for
// running batches, then sets it up on the host (one set-up at a time; it is
// OpenMP-parallel itself) and uploads it.  A request larger than the whole
// budget is refused with CMG_ENOMEM before its set-up.  The batch is solved by one multi-column PCG on the slot's
// stream: every V-cycle launch carries all requests of the batch, requests
// that arrive while others run join the next batch, and batches of different
// slots overlap on the device.  A batch of one request is joined by single
// queued requests of other geometries with the same lattice shape (dimension,
// degree, levels, coarse mesh, box, precision, tolerance and iteration limit)
// whose hierarchies are resident and idle, up to 8 problems: they are solved
// by one grouped PCG (cmg_group_solve), whose V-cycle steps are one launch over
// all of them; groups stay cached while their members are resident.  The
// column arithmetic of the multi-column solve does not depend on the other
// columns, and a grouped solve equals the one-column solve of each member, so
// a result is the same alone and in any batch, group or mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/cutmg.h"
#include "kernels.h"

namespace {

constexpr size_t kBatch = 8;  // requests per multi-column solve (cmg_solve_multi takes up to 8 columns)
constexpr size_t kGroup = 8;  // problems per grouped solve (cmg_group_create takes up to 8)

struct OwnedRequest {
  uint64_t ticket = 0;
  int dim = 0;
  std::vector<double> centers, semi;
  double box_lo = 0, box_hi = 0;
  cmg_params params{};
  std::vector<int> kappa;
  std::vector<double> amp, phase;
  double rtol = 1e-8;
  int maxit = 200;
  double t_submit = 0;
  // the hierarchy's identity, field by field (no struct padding bytes)
  std::string key() const {
    std::string k;
    auto put = [&k](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    auto put_i = [&put](int v) { put(&v, sizeof v); };
    auto put_d = [&put](double v) { put(&v, sizeof v); };
    put_i(dim);
    put_i(static_cast<int>(centers.size()));
    put(centers.data(), centers.size() * sizeof(double));
    put(semi.data(), semi.size() * sizeof(double));
    put_d(box_lo);
    put_d(box_hi);
    const cmg_params& q = params;
    put_i(q.k);
    put_i(q.n_levels);
    put_i(q.coarse_cells);
    put_d(q.gamma_D);
    put_d(q.gamma_g);
    put_i(q.ghost_exp_mode);
    put_i(q.n_c);
    put_i(q.quad_n);
    put_i(q.precond_fp32);
    for (double g : q.gamma_m) put_d(g);
    return k;
  }
  // requests of different geometries that can share one grouped solve
  std::string shape_key() const {
    std::string k;
    auto put = [&k](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    put(&dim, sizeof dim);
    put(&box_lo, sizeof box_lo);
    put(&box_hi, sizeof box_hi);
    put(&params.k, sizeof params.k);
    put(&params.n_levels, sizeof params.n_levels);
    put(&params.coarse_cells, sizeof params.coarse_cells);
    put(&params.precond_fp32, sizeof params.precond_fp32);
    put(&rtol, sizeof rtol);
    put(&maxit, sizeof maxit);
    return k;
  }
  // requests that can share one multi-column solve
  std::string batch_key() const {
    std::string k = key();
    k.append(reinterpret_cast<const char*>(&rtol), sizeof rtol);
    k.append(reinterpret_cast<const char*>(&maxit), sizeof maxit);
    return k;
  }
};

struct Done {
  cmg_result res{};
  std::vector<double> x;
};

struct Entry {
  std::string key;
  cmg_problem* p = nullptr;
  size_t bytes = 0;
  bool in_use = false;
  uint64_t last_use = 0;
  double* db = nullptr;  // right-hand sides and solutions of one batch (kBatch columns), kept with the hierarchy
  double* dx = nullptr;
  int64_t n = 0;         // finest-level DoFs
};

void free_entry(Entry& e) {
  std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());  // no graph capture meanwhile
  cmg_destroy(e.p);  // synchronises the device before freeing
  if (e.db) (void)hipFree(e.db);
  if (e.dx) (void)hipFree(e.dx);
  e.p = nullptr;
  e.db = e.dx = nullptr;
}

}  // namespace

struct cmg_server {
  struct CachedGroup {
    std::vector<std::string> keys;  // the members' hierarchy keys, in member order
    cmg_group* g = nullptr;
  };
  size_t budget = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<OwnedRequest> queue;
  std::map<uint64_t, Done> done;
  std::list<Entry> cache;
  std::set<std::string> pending;  // hierarchies being set up
  std::map<std::string, CachedGroup> groups;  // by the members' keys, concatenated in member order
  size_t used = 0;
  uint64_t next_ticket = 1, use_clock = 0;
  bool stop = false;
  std::mutex setup_mu;  // one host set-up at a time
  std::vector<std::thread> workers;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void finish(cmg_server* S, const OwnedRequest& rq, cmg_result res, std::vector<double>&& x) {
  res.t_done = S->now();
  std::lock_guard<std::mutex> lk(S->mu);
  Done& d = S->done[rq.ticket];
  d.res = res;
  d.x = std::move(x);
  S->cv.notify_all();
}

// Acquire a resident hierarchy for the request: a cached idle one, or a new one
// set up on the host and admitted when its footprint fits into the budget.
cmg_status acquire(cmg_server* S, const OwnedRequest& rq, Entry** out, cmg_result& res) {
  const std::string key = rq.key();
  {
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
      Entry* hit = nullptr;
      bool busy = false;
      for (Entry& e : S->cache)
        if (e.key == key) {
          if (!e.in_use) hit = &e;
          else busy = true;
        }
      if (hit) {
        hit->in_use = true;
        hit->last_use = ++S->use_clock;
        res.cache_hit = 1;
        res.t_admitted = S->now();
        *out = hit;
        return CMG_OK;
      }
      if ((!busy && !S->pending.count(key)) || S->stop) break;
      S->cv.wait(lk);  // the same hierarchy is in use or being set up by another slot
    }
    S->pending.insert(key);
  }
  struct PendingGuard {
    cmg_server* S;
    std::string key;
    ~PendingGuard() {
      std::lock_guard<std::mutex> lk(S->mu);
      S->pending.erase(key);
      S->cv.notify_all();
    }
  } guard{S, key};
  cmg_levelset ls{rq.dim, static_cast<int>(rq.centers.size()) / rq.dim, rq.centers.data(), rq.semi.data(),
                  rq.box_lo, rq.box_hi};
  // admission by footprint before the set-up: counts only, no quadrature or
  // factorisation, so a request that cannot fit costs nothing
  size_t bytes = 0;
  int64_t n = 0;
  cmg_status st = cmg_footprint(&ls, &rq.params, rq.params.precond_fp32 | 2, &bytes, &n);
  if (st != CMG_OK) return st;
  bytes += 2 * kBatch * static_cast<size_t>(n) * sizeof(double);  // the batch's b and x columns
  {
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
      if (S->used + bytes <= S->budget) break;
      // evict the least recently used idle hierarchy
      auto victim = S->cache.end();
      for (auto it = S->cache.begin(); it != S->cache.end(); ++it)
        if (!it->in_use && (victim == S->cache.end() || it->last_use < victim->last_use)) victim = it;
      if (victim != S->cache.end()) {
        S->used -= victim->bytes;
        Entry dead = *victim;
        S->cache.erase(victim);
        // its cached groups go with it (none is in use: that needs every member)
        std::vector<cmg_group*> gone;
        for (auto it = S->groups.begin(); it != S->groups.end();) {
          bool has = false;
          for (const std::string& k : it->second.keys) has = has || k == dead.key;
          if (has) {
            gone.push_back(it->second.g);
            it = S->groups.erase(it);
          } else {
            ++it;
          }
        }
        lk.unlock();
        for (cmg_group* g : gone) cmg_group_destroy(g);
        free_entry(dead);
        lk.lock();
        continue;
      }
      if (S->cache.empty() && S->used == 0) return CMG_ENOMEM;  // larger than the whole budget
      S->cv.wait(lk);  // wait for running solves to release memory
    }
    S->used += bytes;  // reserved for the set-up below
  }
  auto unreserve = [S, bytes]() {
    std::lock_guard<std::mutex> lk(S->mu);
    S->used -= bytes;
    S->cv.notify_all();
  };
  cmg_problem* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->setup_mu);
    st = cmg_setup_host(&ls, &rq.params, &p);
  }
  if (st != CMG_OK) {
    unreserve();
    return st;
  }
  Entry e{key, p, bytes, true, 0, nullptr, nullptr, n};
  st = cmg_upload(p);
  const size_t vb = kBatch * static_cast<size_t>(n) * sizeof(double);
  if (st == CMG_OK) {
    std::lock_guard<std::recursive_mutex> lock(cmg::device_mutex());
    if (hipMalloc(&e.db, vb) != hipSuccess || hipMalloc(&e.dx, vb) != hipSuccess) st = CMG_ENOMEM;
  }
  res.t_admitted = S->now();
  if (st != CMG_OK) {
    free_entry(e);
    unreserve();
    return st;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  e.last_use = ++S->use_clock;
  S->cache.push_back(e);
  *out = &S->cache.back();
  return CMG_OK;
}

void release(cmg_server* S, Entry* e) {
  std::lock_guard<std::mutex> lk(S->mu);
  e->in_use = false;
  S->cv.notify_all();
}

// Right-hand side of one request into bc (n entries) on the worker's stream:
// Fourier loads on the device (the hierarchy's quadrature plan is built at its
// first use and then accounted in the memory in use), the manufactured load on
// the host.
cmg_status load_rhs(cmg_server* S, Entry* e, const OwnedRequest& q, double* bc, int64_t n, hipStream_t stream) {
  if (!q.kappa.empty()) {
    size_t before = 0, after = 0;
    cmg_device_bytes(e->p, 7, &before);
    const cmg_status st = cmg_rhs_fourier_device(e->p, static_cast<int>(q.amp.size()), q.kappa.data(),
                                                 q.amp.data(), q.phase.data(), bc, stream);
    cmg_device_bytes(e->p, 7, &after);
    if (after > before) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->used += after - before;
      e->bytes += after - before;
    }
    return st;
  }
  std::vector<double> B(static_cast<size_t>(n));
  cmg_status st = cmg_rhs_manufactured(e->p, B.data());
  if (st == CMG_OK &&
      (hipMemcpyAsync(bc, B.data(), B.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
       hipStreamSynchronize(stream) != hipSuccess))
    st = CMG_EHIP;
  return st;
}

// Partners of a single request rq whose hierarchy the caller holds: the only
// queued request of each other geometry of rq's lattice shape whose hierarchy
// is resident and idle (taken from the queue, the hierarchy held from here),
// up to kGroup problems in all.  Never waits for a hierarchy.
void take_partners(cmg_server* S, const OwnedRequest& rq, std::vector<OwnedRequest>& partners,
                   std::vector<Entry*>& pe) {
  std::lock_guard<std::mutex> lk(S->mu);
  const std::string sk = rq.shape_key();
  std::unordered_map<std::string, int> count;
  for (const OwnedRequest& q : S->queue)
    if (q.shape_key() == sk) ++count[q.key()];
  std::set<std::string> taken{rq.key()};
  for (auto it = S->queue.begin(); it != S->queue.end() && partners.size() + 1 < kGroup;) {
    Entry* hit = nullptr;
    if (it->shape_key() == sk) {
      const std::string key = it->key();
      if (count[key] == 1 && !taken.count(key) && !S->pending.count(key))
        for (Entry& e : S->cache)
          if (e.key == key && !e.in_use) hit = &e;
    }
    if (!hit) {
      ++it;
      continue;
    }
    hit->in_use = true;
    hit->last_use = ++S->use_clock;
    taken.insert(hit->key);
    pe.push_back(hit);
    partners.push_back(std::move(*it));
    it = S->queue.erase(it);
  }
}

// A single request rq (its hierarchy e0 held, res0 its admission record) with
// partners of other geometries of its lattice shape (their hierarchies pe
// held): one grouped PCG, or one-column solves one after another if the group
// cannot be formed (the members' cut colours differ); the results are the
// same either way.  Releases every hierarchy and finishes every request.
void solve_group(cmg_server* S, OwnedRequest& rq, Entry* e0, const cmg_result& res0,
                 std::vector<OwnedRequest>& partners, std::vector<Entry*>& pe, hipStream_t stream) {
  const int G = 1 + static_cast<int>(partners.size());
  std::vector<OwnedRequest*> req(G);
  req[0] = &rq;
  for (int i = 1; i < G; ++i) req[i] = &partners[i - 1];
  std::vector<cmg_result> res(G);
  const double t_start = S->now();
  for (int i = 0; i < G; ++i) {
    res[i] = cmg_result{};
    res[i].t_submit = req[i]->t_submit;
    res[i].t_start = i == 0 ? res0.t_start : t_start;
    res[i].t_admitted = i == 0 ? res0.t_admitted : t_start;
    res[i].cache_hit = i == 0 ? res0.cache_hit : 1;
    res[i].batch = 1;
    res[i].group = 1;
  }
  std::vector<Entry*> ent(G, nullptr);
  std::vector<cmg_status> st(G, CMG_OK);
  std::vector<int64_t> n(G, 0);
  std::vector<cmg_solve_info> info(G, cmg_solve_info{0, 0.0, 0.0});
  std::vector<std::vector<double>> X(G);
  ent[0] = e0;
  for (int i = 1; i < G; ++i) ent[i] = pe[i - 1];
  for (int i = 0; i < G; ++i) {
    if (!ent[i]) continue;
    cmg_ndofs(ent[i]->p, req[i]->params.n_levels - 1, &n[i]);
    st[i] = load_rhs(S, ent[i], *req[i], ent[i]->db, n[i], stream);
  }
  // the members that reach the solve
  std::vector<int> m;
  for (int i = 0; i < G; ++i)
    if (ent[i] && st[i] == CMG_OK) m.push_back(i);
  const double t_solve = S->now();
  for (int i = 0; i < G; ++i) res[i].t_solve_start = t_solve;
  cmg_group* g = nullptr;
  std::string gk;
  if (m.size() > 1) {
    for (int i : m) gk += ent[i]->key;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->groups.find(gk);
    if (it != S->groups.end()) g = it->second.g;
  }
  if (m.size() > 1 && !g) {
    std::vector<cmg_problem*> ps;
    cmg_server::CachedGroup cg;
    for (int i : m) {
      ps.push_back(ent[i]->p);
      cg.keys.push_back(ent[i]->key);
    }
    if (cmg_group_create(ps.data(), static_cast<int>(ps.size()), &g) == CMG_OK) {
      cg.g = g;
      std::lock_guard<std::mutex> lk(S->mu);
      S->groups[gk] = cg;
    } else {
      g = nullptr;
    }
  }
  if (g) {
    std::vector<const double*> b;
    std::vector<double*> x;
    std::vector<cmg_solve_info> gi(m.size());
    std::vector<cmg_status> gs(m.size(), CMG_OK);
    for (int i : m) {
      b.push_back(ent[i]->db);
      x.push_back(ent[i]->dx);
    }
    (void)cmg_group_solve(g, b.data(), x.data(), rq.rtol, rq.maxit, gi.data(), gs.data(), stream);
    for (size_t j = 0; j < m.size(); ++j) {
      st[m[j]] = gs[j];
      info[m[j]] = gi[j];
      res[m[j]].group = static_cast<int>(m.size());
    }
  } else {
    for (int i : m) st[i] = cmg_solve_multi(ent[i]->p, 1, ent[i]->db, ent[i]->dx, rq.rtol, rq.maxit, &info[i], stream);
  }
  for (int i : m) {
    if (st[i] != CMG_OK && st[i] != CMG_ENOTCONV) continue;
    X[i].resize(static_cast<size_t>(n[i]));
    if (hipMemcpyAsync(X[i].data(), ent[i]->dx, X[i].size() * sizeof(double), hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      st[i] = CMG_EHIP;
  }
  for (int i = 0; i < G; ++i)
    if (ent[i]) release(S, ent[i]);
  for (int i = 0; i < G; ++i) {
    if (st[i] != CMG_OK && st[i] != CMG_ENOTCONV && st[i] != CMG_ENOMEM)
      std::fprintf(stderr, "cutmg server: request of a group of %d failed with status %d: %s\n", G,
                   static_cast<int>(st[i]), cmg_last_error());
    res[i].n_dofs = n[i];
    res[i].info = info[i];
    res[i].status = st[i];
    finish(S, *req[i], res[i], std::move(X[i]));
  }
}

void worker(cmg_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = nullptr;
  (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  for (;;) {
    std::vector<OwnedRequest> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [S] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty()) break;
      batch.push_back(std::move(S->queue.front()));
      S->queue.pop_front();
      const std::string bk = batch[0].batch_key();
      for (auto it = S->queue.begin(); it != S->queue.end() && batch.size() < kBatch;) {
        if (it->batch_key() == bk) {
          batch.push_back(std::move(*it));
          it = S->queue.erase(it);
        } else {
          ++it;
        }
      }
    }
    const int nb = static_cast<int>(batch.size());
    const OwnedRequest& rq = batch[0];
    std::vector<cmg_result> res(nb);
    const double t_start = S->now();
    for (int c = 0; c < nb; ++c) {
      res[c] = cmg_result{};
      res[c].t_submit = batch[c].t_submit;
      res[c].t_start = t_start;
      res[c].batch = nb;
      res[c].group = 1;
    }
    Entry* e = nullptr;
    cmg_status st = acquire(S, rq, &e, res[0]);
    if (nb == 1 && st == CMG_OK) {
      // partners, taken only once the head's hierarchy is held and only if
      // idle (never waited for), so that two slots never wait on each other
      std::vector<OwnedRequest> partners;
      std::vector<Entry*> pe;
      take_partners(S, rq, partners, pe);
      if (!partners.empty()) {
        solve_group(S, batch[0], e, res[0], partners, pe, stream);
        continue;
      }
    }
    for (int c = 1; c < nb; ++c) {
      res[c].cache_hit = res[0].cache_hit;
      res[c].t_admitted = res[0].t_admitted;
    }
    std::vector<double> X;
    int64_t n = 0;
    std::vector<cmg_solve_info> info(nb, cmg_solve_info{0, 0.0, 0.0});
    if (st == CMG_OK) {
      cmg_ndofs(e->p, rq.params.n_levels - 1, &n);
      const size_t bytes = static_cast<size_t>(n) * nb * sizeof(double);
      double* db = e->db;
      double* dx = e->dx;
      for (int c = 0; c < nb && st == CMG_OK; ++c)
        st = load_rhs(S, e, batch[c], db + static_cast<size_t>(c) * n, n, stream);
      const double t_solve = S->now();
      for (int c = 0; c < nb; ++c) res[c].t_solve_start = t_solve;
      if (st == CMG_OK) st = cmg_solve_multi(e->p, nb, db, dx, rq.rtol, rq.maxit, info.data(), stream);
      if (st == CMG_OK || st == CMG_ENOTCONV) {
        X.resize(static_cast<size_t>(n) * nb);
        if (hipMemcpyAsync(X.data(), dx, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
          st = CMG_EHIP;
      }
      release(S, e);
    }
    if (st != CMG_OK && st != CMG_ENOTCONV && st != CMG_ENOMEM)
      std::fprintf(stderr, "cutmg server: batch of %d request(s) failed with status %d: %s\n", nb,
                   static_cast<int>(st), cmg_last_error());
    for (int c = 0; c < nb; ++c) {
      res[c].n_dofs = n;
      res[c].info = info[c];
      // a batch that missed rtol reports it per request
      res[c].status = st == CMG_ENOTCONV ? (info[c].rel_residual <= batch[c].rtol ? CMG_OK : CMG_ENOTCONV) : st;
      std::vector<double> x;
      if (!X.empty()) x.assign(X.begin() + static_cast<size_t>(c) * n, X.begin() + static_cast<size_t>(c + 1) * n);
      finish(S, batch[c], res[c], std::move(x));
    }
  }
  (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

cmg_status cmg_server_create(size_t hbm_budget_bytes, int max_slots, cmg_server** out) {
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes == 0) return CMG_EINVAL;
  auto* S = new cmg_server();
  S->budget = hbm_budget_bytes;
  S->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return CMG_EHIP;
  }
  for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker, S);
  *out = S;
  return CMG_OK;
}

cmg_status cmg_submit(cmg_server* S, const cmg_request* r, uint64_t* ticket) {
  if (!S || !r || !ticket) return CMG_EINVAL;
  const cmg_levelset& ls = r->levelset;
  if (ls.dim < 2 || ls.dim > 3 || ls.n_shapes < 1 || !ls.centers || !ls.semi) return CMG_EINVAL;
  if (r->n_modes < 0 || (r->n_modes > 0 && (!r->kappa || !r->amp || !r->phase))) return CMG_EINVAL;
  OwnedRequest rq;
  rq.dim = ls.dim;
  rq.centers.assign(ls.centers, ls.centers + ls.n_shapes * ls.dim);
  rq.semi.assign(ls.semi, ls.semi + ls.n_shapes * ls.dim);
  rq.box_lo = ls.box_lo;
  rq.box_hi = ls.box_hi;
  rq.params = r->params;
  if (r->n_modes > 0) {
    rq.kappa.assign(r->kappa, r->kappa + r->n_modes * ls.dim);
    rq.amp.assign(r->amp, r->amp + r->n_modes);
    rq.phase.assign(r->phase, r->phase + r->n_modes);
  }
  rq.rtol = r->rtol;
  rq.maxit = r->maxit;
  std::lock_guard<std::mutex> lk(S->mu);
  rq.ticket = S->next_ticket++;
  rq.t_submit = S->now();
  *ticket = rq.ticket;
  S->queue.push_back(std::move(rq));
  S->cv.notify_all();
  return CMG_OK;
}

cmg_status cmg_poll(cmg_server* S, uint64_t ticket, cmg_result* res, double* x_host, int64_t x_len) {
  if (!S || !res) return CMG_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->done.find(ticket);
  if (it == S->done.end()) return CMG_PENDING;
  *res = it->second.res;
  if (x_host) {
    if (x_len != static_cast<int64_t>(it->second.x.size())) return CMG_EINVAL;
    std::memcpy(x_host, it->second.x.data(), it->second.x.size() * sizeof(double));
  }
  S->done.erase(it);
  return CMG_OK;
}

void cmg_server_destroy(cmg_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  for (std::thread& t : S->workers) t.join();
  for (auto& kv : S->groups) cmg_group_destroy(kv.second.g);
  for (Entry& e : S->cache) free_entry(e);
  delete S;
}

}  // extern "C"
