// Continuous-batching engine (internal C++ interface, hz_api.hip): one
// context whose slots are grouped in lanes of equal width; a lane holds the
// right-hand sides of one (request, frequency) pair, with the request's own
// slowness model. Requests on one grid shape join the running BiCGSTAB batch
// between iterations as lanes free up, and leave it when all their right-hand
// sides have stopped.
#pragma once

#include "hz.h"

#include <functional>
#include <vector>

struct hz_engine;

namespace hz {

// One solve request in an engine (every pointer stays valid until done()).
struct EngineJob {
  long long tag;
  const double* m_dev;  // slowness [nz][nx]
  int nfreq;
  std::vector<double> freq_hz;
  double alpha;
  int nrhs;  // per frequency; each frequency takes ceil(nrhs / width) lanes
  const hz_c128* b_dev;
  hz_c128* u_dev;
};

struct EngineHooks {
  // Between iterations: may move jobs into `admit` (at most free_lanes lanes
  // in total; a job takes nfreq * ceil(nrhs / width) of them). `idle`: nothing is running, so the call may
  // wait for work. Returns false to stop the engine (once it is idle).
  std::function<bool(int free_lanes, bool idle, std::vector<EngineJob>& admit)> next;
  // A job has finished: its u_dev is written; info has nfreq * nrhs records.
  std::function<void(long long tag, int rc, std::vector<hz_rhs_info>& info)> done;
};

// Engine over grid (nz, nx) at spacing h with `lanes` lanes of `width` slots,
// BiCGSTAB with the multigrid preconditioner of opts (its tol, maxit, shift,
// smoothing, coarse policy). Ordered on `stream` of `device`.
int engine_create(hz_engine** out, int device, void* stream, int nz, int nx, double h, int lanes, int width,
                  const hz_solve_opts* opts);
void engine_destroy(hz_engine* e);
// Device bytes an engine of this shape holds (all its buffers).
size_t engine_bytes(int nz, int nx, int lanes, int width, const hz_solve_opts* opts);
// Device bytes the engine has allocated.
size_t engine_allocated(const hz_engine* e);
// Runs until hooks.next returns false while idle. Returns HZ_OK or an error
// (jobs running at an error are reported to done() with that error).
int engine_run(hz_engine* e, EngineHooks& hooks);
const char* engine_error(const hz_engine* e);

}  // namespace hz
