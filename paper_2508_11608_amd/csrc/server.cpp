// Continuous-batching solve server on one GPU.
//
// Requests (a level-set domain, discretisation parameters, a right-hand side and
// a tolerance) are queued in arrival order.  Every slot is a worker thread with
// its own HIP stream (default priority).  A slot takes the next request, looks
// for a resident hierarchy with the same geometry and parameters, otherwise
// sets one up on the host (one set-up at a time; it is OpenMP-parallel
// itself) and admits it to the device once its exact footprint fits into the
// HBM budget, evicting least-recently used idle hierarchies.  It then solves
// with V-cycle-preconditioned CG on its own stream, so requests that arrive
// while others run are admitted as slots and memory free up and their kernels
// overlap on the device.  Each solve is deterministic and touches only its own
// hierarchy and vectors, so a result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <chrono>
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
#include <vector>

#include "../../include/cutmg.h"

namespace {

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
  std::string key() const {
    std::string k;
    auto put = [&k](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    put(&dim, sizeof dim);
    put(centers.data(), centers.size() * sizeof(double));
    put(semi.data(), semi.size() * sizeof(double));
    put(&box_lo, sizeof box_lo);
    put(&box_hi, sizeof box_hi);
    put(&params, sizeof params);
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
};

}  // namespace

struct cmg_server {
  size_t budget = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<OwnedRequest> queue;
  std::map<uint64_t, Done> done;
  std::list<Entry> cache;
  std::set<std::string> pending;  // hierarchies being set up
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
  cmg_problem* p = nullptr;
  cmg_status st;
  {
    std::lock_guard<std::mutex> lk(S->setup_mu);
    st = cmg_setup_host(&ls, &rq.params, &p);
  }
  if (st != CMG_OK) return st;
  size_t bytes = 0;
  cmg_device_bytes(p, rq.params.precond_fp32, &bytes);
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
        cmg_problem* vp = victim->p;
        S->cache.erase(victim);
        lk.unlock();
        cmg_destroy(vp);
        lk.lock();
        continue;
      }
      if (S->cache.empty() && S->used == 0) {  // larger than the whole budget
        cmg_destroy(p);
        return CMG_ENOMEM;
      }
      S->cv.wait(lk);  // wait for running solves to release memory
    }
    S->used += bytes;
    S->cache.push_back(Entry{key, p, bytes, true, ++S->use_clock});
    *out = &S->cache.back();
  }
  st = cmg_upload(p);
  res.t_admitted = S->now();
  if (st != CMG_OK) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->used -= bytes;
    for (auto it = S->cache.begin(); it != S->cache.end(); ++it)
      if (&*it == *out) {
        S->cache.erase(it);
        break;
      }
    cmg_destroy(p);
    S->cv.notify_all();
    return st;
  }
  return CMG_OK;
}

void release(cmg_server* S, Entry* e) {
  std::lock_guard<std::mutex> lk(S->mu);
  e->in_use = false;
  S->cv.notify_all();
}

void worker(cmg_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = nullptr;
  (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  for (;;) {
    OwnedRequest rq;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [S] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty()) break;
      rq = std::move(S->queue.front());
      S->queue.pop_front();
    }
    cmg_result res{};
    res.t_submit = rq.t_submit;
    res.t_start = S->now();
    Entry* e = nullptr;
    cmg_status st = acquire(S, rq, &e, res);
    std::vector<double> x;
    if (st == CMG_OK) {
      int64_t n = 0;
      cmg_ndofs(e->p, rq.params.n_levels - 1, &n);
      res.n_dofs = n;
      std::vector<double> b(n);
      st = rq.kappa.empty() ? cmg_rhs_manufactured(e->p, b.data())
                            : cmg_rhs_fourier(e->p, static_cast<int>(rq.amp.size()), rq.kappa.data(), rq.amp.data(),
                                              rq.phase.data(), b.data());
      double *db = nullptr, *dx = nullptr;
      if (st == CMG_OK && (hipMalloc(&db, n * sizeof(double)) != hipSuccess ||
                           hipMalloc(&dx, n * sizeof(double)) != hipSuccess))
        st = CMG_ENOMEM;
      if (st == CMG_OK &&
          hipMemcpyAsync(db, b.data(), n * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess)
        st = CMG_EHIP;
      res.t_solve_start = S->now();
      if (st == CMG_OK) st = cmg_solve(e->p, db, dx, rq.rtol, rq.maxit, &res.info, stream);
      if (st == CMG_OK || st == CMG_ENOTCONV) {
        x.resize(n);
        if (hipMemcpyAsync(x.data(), dx, n * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
          st = CMG_EHIP;
      }
      if (db) (void)hipFree(db);
      if (dx) (void)hipFree(dx);
      release(S, e);
    }
    res.status = st;
    finish(S, rq, res, std::move(x));
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
  for (Entry& e : S->cache) cmg_destroy(e.p);
  delete S;
}

}  // extern "C"
