// Continuous-batching solve server: requests (each a model, a grid, its
// frequencies and right-hand sides) are admitted while their device memory
// footprint fits the budget and an execution slot is free; every slot owns a
// library context and its own HIP stream, so admitted requests run on the
// device at the same time. A slot keeps its context (level hierarchy, Krylov
// and multigrid workspace) allocated from one request to the next, so steady
// state serving allocates nothing. Results do not depend on what else runs:
// every kernel reduction is in a fixed order per right-hand side.

#include "hz.h"
#include "hz_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  long long id = 0;
  hz_request rq{};
  std::vector<double> freqs;
  hz_solve_opts opts{};
  std::vector<double> wlevel;
  size_t footprint = 0;
  Clock::time_point t_submit, t_start, t_end;
  int rc = 0;
  std::vector<hz_rhs_info> info;
  bool done = false;
};

int levels_of(int dim, int nz, int nx, int requested) {
  if (dim == 1) nz = 1;
  const int L = hz::grid_max_levels(dim, nz, nx);
  return requested > 0 ? std::min(requested, L) : hz::grid_default_levels(dim, nz, nx);
}

}  // namespace

struct hz_server {
  int device = 0;
  size_t budget = 0;
  size_t resident_total = 0;       // device memory held by all slots' contexts
  std::vector<size_t> resident;    // per slot
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::deque<Request*> queue;
  std::map<long long, Request*> all;
  long long next_id = 1;
  bool stopping = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  int running = 0, peak_running = 0;
};

namespace {

// A slot's context keeps the memory of the largest request it has served
// (its "resident" footprint). A slot may take the head of the queue when the
// memory of all slots, with its own grown to that request's footprint, fits
// the budget; an idle slot whose memory keeps the head from fitting releases
// it (destroys and recreates its context). A request's footprint never
// exceeds the budget, so the head always fits once the other slots are idle
// and have released their memory.
void worker_loop(hz_server* s, int k) {
  (void)hipSetDevice(s->device);
  hz_ctx* ctx = nullptr;
  const hz_ctx_opts co{s->device, s->streams[k], 0};
  if (hz_create(&ctx, &co) != HZ_OK) ctx = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->stopping && s->queue.empty()) break;
    Request* r = nullptr;
    if (!s->queue.empty()) {
      Request* head = s->queue.front();
      const size_t mine = s->resident[k];
      const size_t grown = std::max(mine, head->footprint);
      if (s->resident_total - mine + grown <= s->budget) {
        r = head;
        s->queue.pop_front();
        s->resident_total += grown - mine;
        s->resident[k] = grown;
      } else if (mine > 0) {
        s->resident_total -= mine;
        s->resident[k] = 0;
        lk.unlock();
        if (ctx) hz_destroy(ctx);
        ctx = nullptr;
        if (hz_create(&ctx, &co) != HZ_OK) ctx = nullptr;
        lk.lock();
        s->cv_work.notify_all();
        continue;
      }
    }
    if (!r) {
      s->cv_work.wait(lk);
      continue;
    }
    s->running += 1;
    s->peak_running = std::max(s->peak_running, s->running);
    r->t_start = Clock::now();
    lk.unlock();
    s->cv_work.notify_all();  // the next request may fit as well
    int rc = HZ_ERR_DEVICE;
    if (ctx) {
      const hz_request& q = r->rq;
      rc = hz_set_model(ctx, q.dim, q.nz, q.nx, q.h, q.m_dev);
      if (rc == HZ_OK) {
        r->opts.jacobi_w_level = r->wlevel.empty() ? nullptr : r->wlevel.data();
        rc = hz_solve(ctx, &r->opts, q.nfreq, r->freqs.data(), q.alpha, q.nrhs, q.b_dev, q.u_dev, r->info.data());
      }
    }
    lk.lock();
    r->rc = rc;
    r->t_end = Clock::now();
    r->done = true;
    s->running -= 1;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  lk.unlock();
  if (ctx) hz_destroy(ctx);
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
  bytes += (size_t)hz::kFineVectors * slots * n[0] * z;         // Krylov and smoothing vectors
  bytes += slots * hz::kShadowMax * (sizeof(int) + z);          // sparse shadow residuals
  for (int l = 1; l < L; ++l) bytes += 4 * slots * n[l] * z;     // level vectors
  if (o->precond == HZ_PRECOND_MG) {
    for (int l = 0; l + 1 < L; ++l) bytes += (size_t)nfreq * n[l] * z;  // tabulated w / diag(M)
    bytes += 2 * (size_t)nfreq * n[L - 1] * n[L - 1] * z;              // coarse inverse and its work copy
  }
  if (o->krylov == HZ_GMRES) bytes += (size_t)(o->gmres_m + 1) * slots * n[0] * z;
  bytes += slots * (sizeof(hz::Slot) + 64) + slots * n[0] / 64 * 4 * sizeof(double);  // reductions
  return bytes;
}

int hz_server_create(hz_server** out, const hz_server_opts* o) {
  if (!out || !o || o->slots < 1 || o->slots > 64) return HZ_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev) return HZ_ERR_ARG;
  hz_server* s = new hz_server();
  s->device = o->device;
  s->budget = o->hbm_budget_bytes ? o->hbm_budget_bytes : (size_t)-1;
  s->resident.assign(o->slots, 0);
  (void)hipSetDevice(s->device);
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
  r->footprint = hz_footprint(rq->dim, rq->nz, rq->nx, rq->nfreq, rq->nrhs, &r->opts);
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
    if (it == s->all.end()) return HZ_ERR_ARG;
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->all.erase(it);
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
