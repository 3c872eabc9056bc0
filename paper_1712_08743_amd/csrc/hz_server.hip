// Continuous-batching solve server. Requests (each a model, a grid, its
// frequencies and right-hand sides) that the batched BiCGSTAB path can take
// (2D, the multigrid preconditioner) are grouped by grid and solver options:
// one engine per group runs all of its requests in one batch, and requests
// that arrive while it runs join the batch between iterations as soon as
// lanes free up (each request keeps its own slowness model and frequencies).
// Engines of different groups, and requests the engines cannot take, run on
// workers of their own, each with its own HIP stream, so their work overlaps
// on the device. Device memory is admitted by footprint against the budget.
// Results do not depend on what else runs: every kernel reduction is in a
// fixed order per right-hand side.

#include "hz.h"
#include "hz_engine.h"
#include "hz_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kLaneWidth = 8;   // right-hand sides per engine lane
constexpr int kMaxLanes = 256;  // lanes of one engine at most
constexpr int kMinLanes = 32;   // lanes an engine is given at least (memory permitting)
// how long an idle engine waits for a request of its group before it gives its memory back
constexpr std::chrono::milliseconds kIdleWait{250};

struct Request {
  long long id = 0;
  hz_request rq{};
  std::vector<double> freqs;
  hz_solve_opts opts{};
  std::vector<double> wlevel;
  size_t footprint = 0;
  std::string group;  // engine group; empty: solved on its own
  int lanes = 0;      // lanes it takes in an engine
  Clock::time_point t_submit, t_start, t_end;
  int rc = 0;
  std::vector<hz_rhs_info> info;
  bool done = false;
  bool claimed = false;  // a waiter holds it
};

int levels_of(int dim, int nz, int nx, int requested) {
  if (dim == 1) nz = 1;
  const int L = hz::grid_max_levels(dim, nz, nx);
  return requested > 0 ? std::min(requested, L) : hz::grid_default_levels(dim, nz, nx);
}

// The engine group of a request: every option the batched solve depends on,
// with the grid; empty when the request cannot be batched.
std::string group_of(const hz_request& rq, const hz_solve_opts& o) {
  if (rq.dim != 2 || o.krylov != HZ_BICGSTAB || o.precond != HZ_PRECOND_MG || o.plain || o.graphs ||
      o.jacobi_w_level || o.restart_at)
    return std::string();
  if (rq.nz < 5 || rq.nx < 5) return std::string();
  char buf[512];
  snprintf(buf, sizeof buf, "%d %d %.17g | %.17g %d %.17g %.17g %d %d %d %.17g %d %d %d %d", rq.nz, rq.nx, rq.h, o.tol,
           o.maxit, o.beta1, o.beta2, o.levels, o.nu1, o.nu2, o.jacobi_w, o.coarse, o.coarse_sweeps, o.autotune,
           o.chunk_rows);
  return std::string(buf);
}

}  // namespace

struct hz_server {
  int device = 0;
  size_t budget = 0;
  size_t resident_total = 0;  // device memory held by running engines and solves
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::deque<Request*> queue;
  std::map<long long, Request*> all;
  std::map<std::string, int> engines;  // groups with a running engine
  long long next_id = 1;
  bool stopping = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  int running = 0, peak_running = 0;
};

namespace {

void finish_request(hz_server* s, Request* r, int rc) {
  r->rc = rc;
  r->t_end = Clock::now();
  r->done = true;
  s->running -= 1;
  s->cv_done.notify_all();
}

void start_request(hz_server* s, Request* r) {
  r->t_start = Clock::now();
  s->running += 1;
  s->peak_running = std::max(s->peak_running, s->running);
}

// Runs one engine for `group` (first request r0, already taken off the
// queue) until it is idle and no request of its group has arrived for a
// short while. Called and returns with the lock held.
void run_engine(hz_server* s, int k, std::unique_lock<std::mutex>& lk, Request* r0, int lanes, size_t bytes) {
  const std::string group = r0->group;
  const hz_request q0 = r0->rq;
  const hz_solve_opts opts = r0->opts;
  std::vector<Request*> first{r0};
  std::map<long long, Request*> inflight;
  lk.unlock();
  hz_engine* e = nullptr;
  int rc = hz::engine_create(&e, s->device, s->streams[k], q0.nz, q0.nx, q0.h, lanes, kLaneWidth, &opts);
  lk.lock();
  if (rc != HZ_OK) {
    start_request(s, r0);
    finish_request(s, r0, rc);
    return;
  }
  // what the engine holds (bytes_in_use reports it; the estimate reserved it)
  const size_t actual = hz::engine_allocated(e);
  s->resident_total = s->resident_total - bytes + actual;
  auto job_of = [&](Request* r) {
    hz::EngineJob jb;
    jb.tag = r->id;
    jb.m_dev = r->rq.m_dev;
    jb.nfreq = r->rq.nfreq;
    jb.freq_hz = r->freqs;
    jb.alpha = r->rq.alpha;
    jb.nrhs = r->rq.nrhs;
    jb.b_dev = r->rq.b_dev;
    jb.u_dev = r->rq.u_dev;
    return jb;
  };
  hz::EngineHooks hooks;
  hooks.next = [&](int free_lanes, bool idle, std::vector<hz::EngineJob>& admit) {
    std::unique_lock<std::mutex> l2(s->mu);
    for (Request* r : first) {
      start_request(s, r);
      inflight[r->id] = r;
      admit.push_back(job_of(r));
      free_lanes -= r->lanes;
    }
    first.clear();
    const auto idle_until = Clock::now() + kIdleWait;
    for (;;) {
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* r = *it;
        if (r->group == group && r->lanes <= free_lanes) {
          it = s->queue.erase(it);
          start_request(s, r);
          inflight[r->id] = r;
          admit.push_back(job_of(r));
          free_lanes -= r->lanes;
        } else {
          ++it;
        }
      }
      if (!admit.empty() || !idle || s->stopping || Clock::now() >= idle_until) break;
      // idle: wait a while for another request of this group before giving the memory back
      s->cv_work.wait_until(l2, idle_until);
    }
    return !(idle && admit.empty());
  };
  hooks.done = [&](long long tag, int jrc, std::vector<hz_rhs_info>& info) {
    std::lock_guard<std::mutex> l2(s->mu);
    auto it = inflight.find(tag);
    if (it == inflight.end()) return;
    Request* r = it->second;
    inflight.erase(it);
    if (!info.empty()) r->info = info;
    finish_request(s, r, jrc);
  };
  lk.unlock();
  rc = hz::engine_run(e, hooks);
  hz::engine_destroy(e);
  lk.lock();
  for (auto& kv : inflight) finish_request(s, kv.second, rc != HZ_OK ? rc : HZ_ERR_DEVICE);
  for (Request* r : first) {
    start_request(s, r);
    finish_request(s, r, rc != HZ_OK ? rc : HZ_ERR_DEVICE);
  }
  s->resident_total = s->resident_total - actual + bytes;  // the caller releases the reservation
}

// One request the engines cannot take, on a context of its own (created and
// released around it, so its memory is exactly its footprint while it runs).
void run_single(hz_server* s, int k, std::unique_lock<std::mutex>& lk, Request* r) {
  start_request(s, r);
  lk.unlock();
  hz_ctx* ctx = nullptr;
  const hz_ctx_opts co{s->device, s->streams[k], 0};
  int rc = hz_create(&ctx, &co);
  if (rc == HZ_OK) {
    const hz_request& q = r->rq;
    rc = hz_set_model(ctx, q.dim, q.nz, q.nx, q.h, q.m_dev);
    if (rc == HZ_OK) {
      r->opts.jacobi_w_level = r->wlevel.empty() ? nullptr : r->wlevel.data();
      rc = hz_solve(ctx, &r->opts, q.nfreq, r->freqs.data(), q.alpha, q.nrhs, q.b_dev, q.u_dev, r->info.data());
    }
    hz_destroy(ctx);
  }
  lk.lock();
  finish_request(s, r, rc);
}

void worker_loop(hz_server* s, int k) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->stopping && s->queue.empty()) break;
    // the first queued request this worker can start: a group without an
    // engine (this worker becomes its engine), or a request on its own
    Request* pick = nullptr;
    int lanes = 0;
    size_t bytes = 0;
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
      Request* r = *it;
      const size_t room = s->budget - s->resident_total;
      if (r->group.empty()) {
        if (r->footprint <= room) {
          pick = r;
          bytes = r->footprint;
          s->queue.erase(it);
          break;
        }
        continue;
      }
      if (s->engines.count(r->group)) continue;  // its engine takes it
      const size_t per_lane = hz::engine_bytes(r->rq.nz, r->rq.nx, 1, kLaneWidth, &r->opts);
      // lanes for twice what the group has queued (at least kMinLanes), within
      // half of the free memory (so that other groups find room), and at
      // least this request's lanes
      long long queued = 0;
      for (const Request* q : s->queue)
        if (q->group == r->group) queued += q->lanes;
      long long want = std::max<long long>(kMinLanes, 2 * queued);
      want = std::min<long long>(want, (long long)((room / 2) / std::max<size_t>(per_lane, 1)));
      want = std::min<long long>(want, kMaxLanes);
      want = std::max<long long>(want, r->lanes);
      const size_t need = hz::engine_bytes(r->rq.nz, r->rq.nx, (int)want, kLaneWidth, &r->opts);
      if (need <= room) {
        pick = r;
        lanes = (int)want;
        bytes = need;
        s->queue.erase(it);
        break;
      }
    }
    if (!pick) {
      s->cv_work.wait(lk);
      continue;
    }
    s->resident_total += bytes;
    // (a finished request may be freed by its waiter at once: nothing of it is read afterwards)
    const std::string group = pick->group;
    if (group.empty()) {
      run_single(s, k, lk, pick);
    } else {
      s->engines[group] = k;
      run_engine(s, k, lk, pick, lanes, bytes);
      s->engines.erase(group);
    }
    s->resident_total -= bytes;
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

size_t hz_footprint(int dim, int nz, int nx, int nfreq, int nrhs, const hz_solve_opts* o) {
  if ((dim != 1 && dim != 2) || nx < 3 || nfreq < 1 || nrhs < 1) return 0;
  if (dim == 1) nz = 1;
  hz_solve_opts d;
  if (!o) {
    hz_default_opts(&d);
    o = &d;
  }
  const size_t z = sizeof(hz_c128);
  const size_t slots = (size_t)nfreq * nrhs;
  const int L = o->precond == HZ_PRECOND_MG ? levels_of(dim, nz, nx, o->levels) : 1;
  size_t n[HZ_MAX_LEVELS];
  int cz = nz, cx = nx;
  for (int l = 0; l < L; ++l) {
    n[l] = (size_t)cz * cx;
    cx = hz::coarse_n(cx);
    if (dim == 2) cz = hz::coarse_n(cz);
  }
  size_t bytes = 0;
  for (int l = 0; l < L; ++l) bytes += n[l] * sizeof(double);  // slowness per level
  bytes += (size_t)hz::kFineVectors * slots * hz::fine_nodes(dim, nz, 1, nx) * z;  // Krylov and smoothing vectors
  bytes += slots * hz::kShadowMax * (sizeof(int) + z);          // sparse shadow residuals
  for (int l = 1; l < L; ++l) bytes += 4 * slots * n[l] * z;     // level vectors
  if (o->precond == HZ_PRECOND_MG) {
    for (int l = 0; l + 1 < L; ++l) bytes += (size_t)nfreq * n[l] * z;  // tabulated w / diag(M)
    bytes += 2 * (size_t)nfreq * n[L - 1] * n[L - 1] * z;              // coarse inverse and its work copy
  }
  if (o->krylov == HZ_GMRES) {
    const size_t m1 = (size_t)o->gmres_m + 1;
    bytes += m1 * slots * n[0] * z;                                                          // basis
    const size_t tiles = (size_t)std::max(hz::vec_tiles(n[0]), hz::gm_dot_tiles(n[0]));
    bytes += slots * tiles * (4 * m1 + 4) * sizeof(double);                                  // partial sums
    bytes += slots * ((2 * m1 * o->gmres_m + 3 * m1 + 2 * (size_t)o->gmres_m) * z +          // small matrices
                      (size_t)o->gmres_m * sizeof(double));                                   // and rotations
  }
  bytes += slots * (sizeof(hz::Slot) + 64) + slots * n[0] / 64 * 4 * sizeof(double);  // reductions
  return bytes;
}

size_t hz_server_footprint(int dim, int nz, int nx, int nfreq, int nrhs, const hz_solve_opts* o) {
  if ((dim != 1 && dim != 2) || nx < 3 || nfreq < 1 || nrhs < 1) return 0;
  hz_solve_opts d;
  if (!o) {
    hz_default_opts(&d);
    o = &d;
  }
  hz_request rq{};
  rq.dim = dim;
  rq.nz = dim == 1 ? 1 : nz;
  rq.nx = nx;
  const long long lanes = (long long)nfreq * ((nrhs + kLaneWidth - 1) / kLaneWidth);
  if (group_of(rq, *o).empty() || lanes > kMaxLanes) return hz_footprint(dim, nz, nx, nfreq, nrhs, o);
  return hz::engine_bytes(nz, nx, (int)lanes, kLaneWidth, o);
}

int hz_server_create(hz_server** out, const hz_server_opts* o) {
  if (!out || !o || o->slots < 1 || o->slots > 64) return HZ_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev) return HZ_ERR_ARG;
  hz_server* s = new hz_server();
  s->device = o->device;
  (void)hipSetDevice(s->device);
  s->budget = o->hbm_budget_bytes;
  if (!s->budget) {  // no limit given: most of the device's free memory
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return HZ_ERR_DEVICE;
    }
    s->budget = fr / 10 * 9;
  }
  for (int k = 0; k < o->slots; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return HZ_ERR_DEVICE;
    }
    s->streams.push_back(st);
  }
  for (int k = 0; k < o->slots; ++k) s->workers.emplace_back(worker_loop, s, k);
  *out = s;
  return HZ_OK;
}

void hz_server_destroy(hz_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

int hz_server_submit(hz_server* s, const hz_request* rq, long long* ticket) {
  if (!s || !rq || !ticket) return HZ_ERR_ARG;
  if (rq->nfreq < 1 || rq->nrhs < 1 || !rq->freq_hz || !rq->b_dev || !rq->u_dev || !rq->m_dev)
    return HZ_ERR_ARG;
  Request* r = new Request();
  r->rq = *rq;
  r->freqs.assign(rq->freq_hz, rq->freq_hz + rq->nfreq);
  if (rq->opts) r->opts = *rq->opts;
  else hz_default_opts(&r->opts);
  if (r->opts.jacobi_w_level) {
    const int L = levels_of(rq->dim, rq->dim == 1 ? 1 : rq->nz, rq->nx, r->opts.levels);
    r->wlevel.assign(r->opts.jacobi_w_level, r->opts.jacobi_w_level + std::max(0, L - 1));
  }
  r->rq.freq_hz = nullptr;
  r->rq.opts = nullptr;
  r->group = group_of(r->rq, r->opts);
  r->lanes = rq->nfreq * ((rq->nrhs + kLaneWidth - 1) / kLaneWidth);
  if (r->lanes > kMaxLanes) r->group.clear();
  r->footprint = r->group.empty() ? hz_footprint(rq->dim, rq->nz, rq->nx, rq->nfreq, rq->nrhs, &r->opts)
                                  : hz::engine_bytes(rq->nz, rq->nx, r->lanes, kLaneWidth, &r->opts);
  if (!r->group.empty() && r->footprint != hz_server_footprint(rq->dim, rq->nz, rq->nx, rq->nfreq, rq->nrhs, &r->opts))
    r->group.clear();  // (the two must agree)
  if (r->footprint == 0 || r->footprint > s->budget) {
    delete r;
    return HZ_ERR_NOMEM;
  }
  r->info.resize((size_t)rq->nfreq * rq->nrhs);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    s->all[r->id] = r;
    s->queue.push_back(r);
  }
  s->cv_work.notify_all();
  *ticket = r->id;
  return HZ_OK;
}

int hz_server_wait(hz_server* s, long long ticket, hz_rhs_info* info, double* times) {
  if (!s) return HZ_ERR_ARG;
  Request* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end() || it->second->claimed) return HZ_ERR_ARG;
    r = it->second;
    r->claimed = true;  // a second waiter on this ticket is refused
    s->cv_done.wait(lk, [&] { return r->done; });
    s->all.erase(ticket);
  }
  if (info) std::copy(r->info.begin(), r->info.end(), info);
  if (times) {
    times[0] = std::chrono::duration<double>(r->t_start - r->t_submit).count();  // queued
    times[1] = std::chrono::duration<double>(r->t_end - r->t_start).count();     // on the device
    times[2] = std::chrono::duration<double>(r->t_end - r->t_submit).count();    // latency
  }
  const int rc = r->rc;
  delete r;
  return rc;
}

int hz_server_stats(hz_server* s, int* queued, int* running, int* peak_running, size_t* bytes_in_use) {
  if (!s) return HZ_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int)s->queue.size();
  if (running) *running = s->running;
  if (peak_running) *peak_running = s->peak_running;
  if (bytes_in_use) *bytes_in_use = s->resident_total;
  return HZ_OK;
}

}  // extern "C"
