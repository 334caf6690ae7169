// Request server of libhmps: continuous batching of power-series solves
// over resident geometries under an HBM budget (host code; the solves run
// in the library's kernels on the server's streams).
//
// Workers: one thread and one HIP stream (default priority) per slot.  A
// free worker takes the oldest queued request whose geometry is not in use
// by another worker, together with every later queued request of the same
// geometry and solve options up to kMaxBatchRhs right-hand sides (columns
// are concatenated into one ps_solve), so requests that arrive while others
// run join the next batch of their geometry, and batches of different
// geometries run at the same time on different streams.
//
// Geometries: built on first use from the problem given with a request
// (host part, then device part on the worker's stream) and kept resident.
// Before a device part is built, least recently used geometries with no
// queued or running request are freed until the resident bytes (blocks and
// workspaces) plus the new geometry's estimate fit the budget.  If they do
// not fit yet: while a resident geometry has queued requests that no
// worker runs, the cold build steps aside (its host part kept) and the
// worker serves those requests first, since they release that geometry;
// while other batches or builds run, the build waits for them; a geometry
// that does not fit an idle device fails its requests with HM_ENOMEM.
// Handles freed to make room are released after the server lock is
// dropped (a free synchronises the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hm_internal.h"
#include "krylov.h"

namespace {

using hm::cplx;
using clk = std::chrono::steady_clock;
constexpr int kMaxBatchRhs = 64;

struct Spec {  // a copy of the problem and build options of a geometry
  std::vector<double> xyz, chi;
  hm_problem prob{};
  hm_build_opts opts{};
};

struct Geometry {
  hm_matrix_t h = nullptr;
  int64_t n = 0;
  int64_t bytes = 0;     // resident device bytes (blocks + workspace)
  bool building = false;
  bool reserved = false; // building, with its device bytes counted
  bool busy = false;     // a worker runs a batch on it
  bool wait_room = false;  // a cold build stepped aside until room frees up
  hm_matrix_t staged = nullptr;  // its host part, kept meanwhile
  int pending = 0;       // queued + running requests
  clk::time_point last_used;
  int64_t builds = 0;
};

struct Request {
  hm_ticket_t id = 0;
  uint64_t key = 0;
  ps_opts opts{};
  int32_t nrhs = 0;
  std::vector<cplx> b, x;
  std::vector<ps_stats> stats;
  int32_t state = PS_QUEUED;
  int status = HM_OK;
  std::string err;
  clk::time_point t_submit, t_done;
  bool cold = false;  // its batch had to build the geometry
};

bool same_opts(const ps_opts& a, const ps_opts& b) {
  return a.K == b.K && a.level == b.level && a.precision == b.precision && a.kind == b.kind &&
         a.max_passes == b.max_passes && a.refine_tol == b.refine_tol &&
         (a.kind != PS_GMRES || a.restart == b.restart);
}

}  // namespace

struct hm_server {
  int device = 0;
  int64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;       // queue or geometry state changed
  std::map<uint64_t, Geometry> geoms;
  std::map<uint64_t, std::shared_ptr<Spec>> specs;
  std::deque<Request*> queue;
  std::unordered_map<hm_ticket_t, std::unique_ptr<Request>> tickets;
  hm_ticket_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  int64_t slot_bytes = 0;           // device staging of the workers
  ps_server_stats st{};

  int64_t resident() const {
    int64_t r = slot_bytes;
    for (auto& kv : geoms) r += kv.second.bytes;
    return r;
  }
  void worker(int slot);
  // with mu held: drop idle geometries (LRU first) until need more bytes
  // fit; their handles go to `freed`, to be released without the lock
  bool make_room(int64_t need, uint64_t except, std::vector<hm_matrix_t>& freed);
  // with mu held: a resident geometry other than `except` with queued
  // requests and no worker on it
  bool runnable_elsewhere(uint64_t except) const {
    for (auto& kv : geoms)
      if (kv.first != except && kv.second.h && !kv.second.busy && !kv.second.building &&
          kv.second.pending > 0)
        return true;
    return false;
  }
  // with mu held: batches or builds (with their room) running elsewhere
  bool running_elsewhere(uint64_t except) const {
    for (auto& kv : geoms)
      if (kv.first != except && (kv.second.busy || kv.second.reserved)) return true;
    return false;
  }
  void finish(std::vector<Request*>& batch, int status, const std::string& err);
};

bool hm_server::make_room(int64_t need, uint64_t except, std::vector<hm_matrix_t>& freed) {
  while (resident() + need > budget) {
    uint64_t victim = 0;
    bool found = false;
    clk::time_point oldest = clk::time_point::max();
    for (auto& kv : geoms) {
      const Geometry& g = kv.second;
      if (kv.first == except || !g.h || g.busy || g.building || g.pending > 0) continue;
      if (g.last_used < oldest) {
        oldest = g.last_used;
        victim = kv.first;
        found = true;
      }
    }
    if (!found) return false;
    Geometry& g = geoms[victim];
    freed.push_back(g.h);
    g.h = nullptr;
    g.bytes = 0;
    st.evictions++;
  }
  return true;
}

void hm_server::finish(std::vector<Request*>& batch, int status, const std::string& err) {
  const auto now = clk::now();
  for (Request* r : batch) {
    r->state = (status == HM_OK || status == HM_EDIVERGED) ? PS_DONE : PS_FAILED;
    r->status = status;
    if (r->state == PS_DONE) {  // a request's own columns decide its status
      r->status = HM_OK;
      for (const auto& q : r->stats)
        if (q.diverged) r->status = HM_EDIVERGED;
    }
    r->err = err;
    r->t_done = now;
    const double ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    for (auto& s : r->stats) s.t_ms = ms;
    std::vector<cplx>().swap(r->b);
    if (r->state == PS_DONE) {
      st.requests_done++;
      st.rhs_done += r->nrhs;
    } else {
      st.requests_failed++;
    }
  }
}

void hm_server::worker(int slot) {
  (void)hipSetDevice(device);
  hipStream_t stream = nullptr;
  (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  // device and pinned host staging, grown to the largest batch seen
  size_t cap = 0;
  void *db = nullptr, *dx = nullptr;
  cplx *hb = nullptr, *hx = nullptr;
  // grown geometrically, so a stream of growing batches reallocates (and
  // synchronises the device in the frees) only a few times
  auto grow = [&](size_t want) -> int {
    if (want <= cap) return HM_OK;
    const size_t elems = std::max(want, 2 * cap);
    const size_t bytes = elems * sizeof(cplx);
    if (db) (void)hipFree(db);
    if (dx) (void)hipFree(dx);
    if (hb) (void)hipHostFree(hb);
    if (hx) (void)hipHostFree(hx);
    db = dx = nullptr;
    hb = hx = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      slot_bytes -= 2 * (int64_t)cap * (int64_t)sizeof(cplx);
    }
    cap = 0;
    if (hipMalloc(&db, bytes) != hipSuccess || hipMalloc(&dx, bytes) != hipSuccess ||
        hipHostMalloc((void**)&hb, bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&hx, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return HM_ENOMEM;
    }
    cap = elems;
    std::lock_guard<std::mutex> lk(mu);
    slot_bytes += 2 * (int64_t)bytes;
    return HM_OK;
  };

  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // ---- pick: oldest request whose geometry is free (or buildable);
    // builds that stepped aside for room come last
    Request* head = nullptr;
    for (int pass = 0; pass < 2 && !head; ++pass)
      for (Request* r : queue) {
        Geometry& g = geoms[r->key];
        if (g.busy || g.building || (pass == 0 && g.wait_room)) continue;
        head = r;
        break;
      }
    if (!head) {
      if (stop) break;
      cv.wait(lk);
      continue;
    }
    const uint64_t key = head->key;
    Geometry& g = geoms[key];
    bool cold = false;
    if (!g.h) {
      // ---- cold geometry: host part, room under the budget, device part
      auto spec = specs[key];
      g.building = true;
      hm_matrix_t h = g.staged;  // host part of an earlier attempt, if any
      g.staged = nullptr;
      lk.unlock();
      int s = HM_OK;
      std::string err;
      if (!h) {
        s = hm::build_host_phase(&spec->prob, &spec->opts, &h);
        if (s != HM_OK) err = hm_last_error();
      }
      const int64_t need = s == HM_OK ? hm::device_bytes_estimate(h, head->nrhs) : 0;
      lk.lock();
      std::vector<hm_matrix_t> freed;
      bool aside = false;
      while (s == HM_OK && !make_room(need, key, freed)) {
        // queued requests of a resident geometry that no worker runs hold
        // it in place: serve them first (they release it), keep the host part
        if (runnable_elsewhere(key)) {
          aside = true;
          break;
        }
        // else wait only for work that will end without this worker:
        // running batches and builds that already hold their room
        if (!running_elsewhere(key)) {
          s = HM_ENOMEM;
          err = "geometry needs about " + std::to_string(need) +
                " device bytes, more than the budget allows";
          break;
        }
        cv.wait(lk);
      }
      if (aside) {
        g.staged = h;
        g.wait_room = true;
        g.building = false;
        lk.unlock();
        for (hm_matrix_t f : freed) hmat_free(f);
        lk.lock();
        cv.notify_all();
        continue;
      }
      g.wait_room = false;
      if (s == HM_OK) {
        g.bytes = need;  // reserved until the real size is known
        g.reserved = true;
        lk.unlock();
        for (hm_matrix_t f : freed) hmat_free(f);
        freed.clear();
        s = hm::build_device_phase(h, &spec->opts, stream);
        if (s == HM_OK && hipStreamSynchronize(stream) != hipSuccess) s = HM_EHIP;
        if (s != HM_OK) err = hm_last_error();
        lk.lock();
      }
      g.building = false;
      g.reserved = false;
      if (!freed.empty()) {
        lk.unlock();
        for (hm_matrix_t f : freed) hmat_free(f);
        freed.clear();
        lk.lock();
      }
      if (s != HM_OK) {
        if (h) hmat_free(h);
        g.bytes = 0;
        std::vector<Request*> failed;
        for (auto it = queue.begin(); it != queue.end();) {
          if ((*it)->key == key) {
            failed.push_back(*it);
            it = queue.erase(it);
          } else {
            ++it;
          }
        }
        g.pending -= (int)failed.size();
        finish(failed, s, "build: " + err);
        cv.notify_all();
        continue;
      }
      g.h = h;
      g.n = hm::matrix_n(h);
      g.bytes = hm::resident_bytes(h);
      g.builds++;
      st.builds++;
      cold = true;
    }
    // ---- batch: head plus later requests of the same geometry and options
    std::vector<Request*> batch;
    int cols = 0;
    const ps_opts o = head->opts;
    for (auto it = queue.begin(); it != queue.end();) {
      Request* r = *it;
      if (r->key == key && same_opts(r->opts, o) &&
          (batch.empty() || cols + r->nrhs <= kMaxBatchRhs)) {
        batch.push_back(r);
        cols += r->nrhs;
        r->state = PS_RUNNING;
        r->cold = cold;
        it = queue.erase(it);
      } else {
        ++it;
      }
    }
    g.busy = true;
    hm_matrix_t h = g.h;
    const int64_t n = g.n;
    st.batches++;
    st.batch_rhs += cols;
    // a wider batch than before grows the geometry's workspace: room first.
    // When no room can be made (the other resident geometries hold queued
    // work and nothing runs that would release memory), the batch is solved
    // in pieces of the width the geometry's workspace already holds.
    int s = HM_OK;
    std::string err;
    std::vector<hm_matrix_t> freed;
    int chunk = cols;
    if (cols > hm::workspace_rhs(h)) {
      const int64_t extra = hm::workspace_bytes(h, cols, 0) - hm::workspace_bytes(h, hm::workspace_rhs(h), 0);
      bool grown = true;
      while (!make_room(extra, key, freed)) {
        if (!running_elsewhere(key)) {
          grown = false;
          if (hm::workspace_rhs(h) >= 1) {
            chunk = hm::workspace_rhs(h);
          } else {
            s = HM_ENOMEM;
            err = "workspace for " + std::to_string(cols) + " right-hand sides exceeds the budget";
          }
          break;
        }
        cv.wait(lk);
      }
      if (grown) g.bytes += extra;
    }
    // GMRES keeps its basis on the handle: room for its growth too
    if (s == HM_OK && o.kind == PS_GMRES) {
      const int m = hm::gmres_restart(o);
      const int64_t extra = hm::gmres_growth_bytes(h, m, chunk);
      bool grown = true;
      while (extra > 0 && !make_room(extra, key, freed)) {
        if (!running_elsewhere(key)) {
          grown = false;
          if (hm::gmres_rhs(h, m) >= 1) {
            chunk = std::min(chunk, hm::gmres_rhs(h, m));
          } else {
            s = HM_ENOMEM;
            err = "GMRES workspace for " + std::to_string(cols) + " right-hand sides exceeds the budget";
          }
          break;
        }
        cv.wait(lk);
      }
      if (grown) g.bytes += extra;
    }
    if (chunk < cols) st.split_batches++;
    lk.unlock();
    for (hm_matrix_t f : freed) hmat_free(f);

    // ---- run: pack b, copy in, solve, copy out
    if (s == HM_OK) {
      s = grow((size_t)n * cols);
      if (s != HM_OK) err = "worker staging allocation failed";
    }
    std::vector<ps_stats> stats(cols);
    bool diverged = false;
    if (s == HM_OK) {
      int c0 = 0;
      for (Request* r : batch) {
        std::memcpy(hb + (size_t)n * c0, r->b.data(), sizeof(cplx) * n * r->nrhs);
        c0 += r->nrhs;
      }
      const size_t bytes = sizeof(cplx) * (size_t)n * cols;
      if (hipMemcpyAsync(db, hb, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) s = HM_EHIP;
      for (int q0 = 0; s == HM_OK && q0 < cols; q0 += chunk) {
        const int qn = std::min(chunk, cols - q0);
        const int sq = ps_solve(h, &o, static_cast<cplx*>(db) + (size_t)n * q0, n,
                                static_cast<cplx*>(dx) + (size_t)n * q0, n, qn, stats.data() + q0, stream);
        if (sq == HM_EDIVERGED) {
          diverged = true;
        } else if (sq != HM_OK) {
          s = sq;
          err = hm_last_error();
        }
      }
      if (s == HM_OK && diverged) s = HM_EDIVERGED;
      if ((s == HM_OK || s == HM_EDIVERGED) &&
          (hipMemcpyAsync(hx, dx, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
           hipStreamSynchronize(stream) != hipSuccess)) {
        s = HM_EHIP;
        err = "copy of the result failed";
      }
      if (s == HM_OK || s == HM_EDIVERGED) {
        c0 = 0;
        for (Request* r : batch) {
          r->x.assign(hx + (size_t)n * c0, hx + (size_t)n * (c0 + r->nrhs));
          r->stats.assign(stats.begin() + c0, stats.begin() + c0 + r->nrhs);
          for (auto& q : r->stats) q.built = r->cold ? 1 : 0;
          c0 += r->nrhs;
        }
      }
    }

    lk.lock();
    g.busy = false;
    g.last_used = clk::now();
    g.pending -= (int)batch.size();
    g.bytes = hm::resident_bytes(h);
    finish(batch, s, err);
    cv.notify_all();
  }
  lk.unlock();
  if (db) (void)hipFree(db);
  if (dx) (void)hipFree(dx);
  if (hb) (void)hipHostFree(hb);
  if (hx) (void)hipHostFree(hx);
  if (stream) (void)hipStreamDestroy(stream);
  (void)slot;
}

extern "C" {

int ps_server_create(size_t hbm_budget_bytes, int32_t max_slots, hm_server_t* out) {
  if (!out) { hm::set_error("null output"); return HM_EINVAL; }
  *out = nullptr;
  if (max_slots < 1 || max_slots > 16) { hm::set_error("max_slots must be in [1, 16]"); return HM_EINVAL; }
  std::unique_ptr<hm_server> s(new hm_server());
  if (hipGetDevice(&s->device) != hipSuccess) { hm::set_error("no device"); return HM_EHIP; }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { hm::set_error("hipMemGetInfo failed"); return HM_EHIP; }
  s->budget = hbm_budget_bytes ? (int64_t)hbm_budget_bytes : (int64_t)(0.9 * (double)free_b);
  s->st.budget_bytes = s->budget;
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(&hm_server::worker, s.get(), i);
  *out = s.release();
  return HM_OK;
}

int ps_submit(hm_server_t s, uint64_t geom_key, const hm_problem* prob, const hm_build_opts* bopts,
              const ps_opts* opts, const void* b_host, int32_t nrhs, hm_ticket_t* out) {
  if (!s || !opts || !out || (nrhs > 0 && !b_host)) { hm::set_error("null argument"); return HM_EINVAL; }
  if (nrhs < 1 || nrhs > kMaxBatchRhs) {
    hm::set_error("nrhs must be in [1, 64]");
    return HM_EINVAL;
  }
  if (opts->K < 0 || opts->K > 10000 ||
      (opts->precision != HM_F64 && opts->precision != HM_F32_APPLY) ||
      (opts->kind != PS_SERIES && opts->kind != PS_REFINE && opts->kind != PS_REFINE_FIXED &&
       opts->kind != PS_GMRES) ||
      (opts->kind != PS_SERIES && (opts->max_passes < 0 || !(opts->refine_tol > 0))) ||
      (opts->kind == PS_GMRES &&
       (opts->max_passes < 1 || opts->restart < 0 || opts->restart > hm::kMaxKrylov))) {
    hm::set_error("bad solve options");
    return HM_EINVAL;
  }
  std::unique_ptr<Request> r(new Request());
  r->key = geom_key;
  r->opts = *opts;
  r->nrhs = nrhs;
  r->t_submit = clk::now();
  std::shared_ptr<Spec> spec;
  if (prob) {
    if (!bopts) { hm::set_error("a new geometry needs build options"); return HM_EINVAL; }
    if (!prob->xyz || prob->n < 1 || (prob->kind == HM_VOLUME && !prob->chi)) {
      hm::set_error("bad problem");
      return HM_EINVAL;
    }
    spec = std::make_shared<Spec>();
    spec->xyz.assign(prob->xyz, prob->xyz + 3 * prob->n);
    if (prob->kind == HM_VOLUME) spec->chi.assign(prob->chi, prob->chi + prob->n);
    spec->prob = *prob;
    spec->prob.xyz = spec->xyz.data();
    spec->prob.chi = spec->chi.empty() ? nullptr : spec->chi.data();
    spec->opts = *bopts;
    spec->opts.progress = nullptr;
    spec->opts.progress_user = nullptr;
    spec->opts.flags &= ~(HM_BUILD_HOST_ONLY | HM_BUILD_KEEP_HOST);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto sp = s->specs.find(geom_key);
  if (sp == s->specs.end()) {
    if (!spec) { hm::set_error("unknown geometry key and no problem given"); return HM_EINVAL; }
    s->specs[geom_key] = spec;
    sp = s->specs.find(geom_key);
  }
  const int64_t n = sp->second->prob.n;
  r->b.assign(static_cast<const cplx*>(b_host), static_cast<const cplx*>(b_host) + n * nrhs);
  r->id = s->next_ticket++;
  *out = r->id;
  Geometry& g = s->geoms[geom_key];
  g.pending++;
  s->queue.push_back(r.get());
  s->tickets[r->id] = std::move(r);
  s->st.requests_submitted++;
  s->cv.notify_all();
  return HM_OK;
}

int ps_poll(hm_server_t s, hm_ticket_t t, void* x_host, ps_stats* per_rhs, int32_t* state) {
  if (!s) { hm::set_error("null server"); return HM_EINVAL; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(t);
  if (it == s->tickets.end()) { hm::set_error("unknown ticket"); return HM_EINVAL; }
  Request* r = it->second.get();
  if (state) *state = r->state;
  if (r->state == PS_QUEUED || r->state == PS_RUNNING) return HM_ENOTREADY;
  int status = r->status;
  if (r->state == PS_DONE) {
    if (x_host) std::memcpy(x_host, r->x.data(), sizeof(cplx) * r->x.size());
    if (per_rhs) std::copy(r->stats.begin(), r->stats.end(), per_rhs);
  } else {
    hm::set_error(r->err);
  }
  if (x_host || per_rhs) s->tickets.erase(it);  // delivered: release
  return status;
}

int ps_server_info(hm_server_t s, ps_server_stats* out) {
  if (!s || !out) { hm::set_error("null argument"); return HM_EINVAL; }
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->resident_bytes = s->resident();
  out->resident_geometries = 0;
  for (auto& kv : s->geoms) out->resident_geometries += kv.second.h ? 1 : 0;
  out->queued = (int64_t)s->queue.size();
  return HM_OK;
}

int ps_server_destroy(hm_server_t s) {
  if (!s) return HM_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Request* r : s->queue) {
      r->state = PS_FAILED;
      r->status = HM_ESTATE;
      r->err = "server destroyed";
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  for (auto& w : s->workers) w.join();
  for (auto& kv : s->geoms) {
    if (kv.second.h) hmat_free(kv.second.h);
    if (kv.second.staged) hmat_free(kv.second.staged);
  }
  delete s;
  return HM_OK;
}

}  // extern "C"
