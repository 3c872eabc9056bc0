// C-ABI of the Helmholtz solver library: context, model, plan, setup of the
// multigrid hierarchy and coarse inverses, and the host drivers of the
// batched Krylov solvers. Device work is enqueued on the context's stream;
// the host only marshals arguments, sizes launches and polls a small summary
// that the device writes into mapped host memory.

#include "hz.h"
#include "hz_engine.h"
#include "hz_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <deque>
#include <string>
#include <vector>
#include <map>
#include <mutex>
#include <array>

using namespace hz;

namespace {

// The allocation-free solve (hz_solve_noalloc) takes its workspace from a
// static device array: while an arena is installed on the calling thread,
// DevBuf::ensure hands out 256-byte aligned regions of it (a bump pointer)
// instead of calling hipMalloc, and such regions are never freed.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  size_t wanted = 0;  // end of the furthest region asked for (above cap: refused)
};
thread_local Arena* t_arena = nullptr;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // a region of the arena, not ours to free
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
  }
  hipError_t ensure(size_t nb) {
    if (nb <= bytes && p) return hipSuccess;
    if (nb == 0) nb = 256;
    if (t_arena) {
      // an owned buffer here would have to be freed: the caller stashes them all first
      if (p && !borrowed) return hipErrorInvalidValue;
      const size_t off = (t_arena->used + 255) & ~(size_t)255;
      t_arena->wanted = std::max(t_arena->wanted, off + nb);
      if (off + nb > t_arena->cap) return hipErrorOutOfMemory;
      p = t_arena->base + off;
      bytes = nb;
      borrowed = true;
      t_arena->used = off + nb;
      return hipSuccess;
    }
    release();
    hipError_t e = hipMalloc(&p, nb);
    if (e == hipSuccess) bytes = nb;
    else p = nullptr;
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Workspace of the allocation-free solve: one array per device, found by
// hipGetSymbolAddress at context creation (the name is only a host-side
// stand-in for it). Every call on a device shares that device's array.
__device__ __align__(256) unsigned char scratch[HZ_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// With the device current: the address of this device's scratch array (looked up once).
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

struct LevelInfo {
  int nz = 0, nx = 0, ny = 1;  // ny > 1 on 3D grids only
  double h = 0.0;
  DevBuf m;
  DevBuf rho;          // density of Eq. (1) on this level (when hz_ctx::has_rho)
  DevBuf dc;           // 2D: its coupling table for the fused kernels (Grid::dc)
  size_t mstride = 0;  // engines: one model per lane, mstride apart (see Grid::mstride)
  size_t n() const { return (size_t)nz * ny * nx; }
  int rows() const { return nz * ny; }  // rows of the 2D tiling of the grid
};

// Fine-level vectors of the solvers (x is the caller's output buffer).
enum FineVec { kR, kRh, kP, kP2, kV, kPh, kPh2, kS, kSh, kSh2, kT, kT1, kT2, kNumFine };
static_assert(kNumFine == kFineVectors, "the footprint counts kFineVectors fine vectors");
// Per coarse level: right-hand side, result, two smoothing buffers.
enum LevelVec { kLb, kLu, kLx, kLy, kNumLevelVec };

constexpr int kRing = 8;
constexpr int kLag = 2;

}  // namespace

struct hz_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  std::string err;
  // model
  int dim = 0, nz = 0, nx = 0, ny = 1;
  // mmin, mmax: the slowness range the V-cycle is planned for (m / sqrt(rho)
  // under a density); m_lo, m_hi: the range of the model itself
  double h = 0.0, mmin = 0.0, mmax = 0.0, m_lo = 0.0, m_hi = 0.0;
  int maxlev = 0;
  int has_rho = 0;  // a density of Eq. (1) is set
  LevelInfo lv[kMaxLevels];
  int model_version = 0;
  // solver workspace (the finest-level vectors hold fine_nodes() nodes per slot)
  DevBuf fine[kNumFine];
  // > 0 while a fused 2D BiCGSTAB solve runs with pitched finest-level vectors:
  // their row pitch (grid_of(c, 0) and level_stride(c, 0) follow it)
  int fine_px = 0;
  DevBuf lev[kMaxLevels][kNumLevelVec];
  int ws_slots = 0, ws_levels = 0;
  DevBuf slots, active, nactive, freqtab, partials, resid, fstart;
  DevBuf rh_idx, rh_val;  // sparse shadow residuals, [slot_cap][kShadowMax]
  int cur_nfreq = 1, cur_nrhs = 1;  // layout of the slots of the current batch
  int partial_tiles = 0;
  int slot_cap = 0;
  // coarse inverses for the current frequencies
  DevBuf cinv_a, cinv_b;
  DevBuf winv;  // w_l / diag(M_l) per frequency and smoothing level
  std::vector<double> cinv_key;  // omega, beta1, beta2 per frequency + levels + version
  const double2* cinv_base = nullptr;
  // small uploads
  DevBuf scratch_int, scratch_c;
  DevBuf misfit_b, misfit_u, misfit_d, misfit_out;
  DevBuf gm_V, gm_small, gm_part;
  DevBuf fwi_b, fwi_u, fwi_mu, fwi_d, fwi_int, fwi_omega, fwi_out;
  DevBuf gn_g, gn_r, gn_p, gn_hp, gn_state;
  // host polling
  Summary* ring_host = nullptr;
  Summary* ring_dev = nullptr;
  hipEvent_t ev[kRing] = {};
  size_t max_lds = 0;
  double wall_khz = 0.0;
  // kernel timing for measurement
  unsigned timing_mask = 0;
  std::vector<hipEvent_t> tpool;   // free events
  struct Pair {
    hipEvent_t a, b;
    int cls;
  };
  std::vector<Pair> tpairs;        // recorded, not yet folded
  long long t_launches[HZ_KERNEL_CLASSES] = {};
  double t_ms[HZ_KERNEL_CLASSES] = {};
  // launch-shape tuning: rows per wavefront of the fused V-cycle kernels,
  // keyed by (kernel, nz, nx, batch-size octave)
  std::map<std::array<int, 4>, int> tuned_chunk;
  hipStream_t graph_stream = nullptr;  // the library's own stream, used only to capture graphs
  bool any_coarse_jacobi = false;      // set by setup_freqs for the running solve
  int tune_mode = 1;   // opts.autotune of the running solve
  int fixed_chunk = 0; // opts.chunk_rows of the running solve
  // inside hz_solve_noalloc: no launch-shape trials, no timing events, no graphs
  bool noalloc = false;
  hipError_t scratch_status = hipSuccess;  // lookup of the device's scratch array at creation
};

namespace {

int fail(hz_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HZ_HIP(c, call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((c), HZ_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

#define HZ_ALLOC(c, buf, bytes)                                                            \
  do {                                                                                     \
    hipError_t e_ = (buf).ensure(bytes);                                                   \
    if (e_ != hipSuccess)                                                                  \
      return fail((c), HZ_ERR_NOMEM, "device allocation of %zu bytes failed: %s",          \
                  (size_t)(bytes), hipGetErrorString(e_));                                 \
  } while (0)

Grid grid_of(const hz_ctx* c, int l) {
  Grid g;
  g.nz = c->lv[l].nz;
  g.nx = c->lv[l].nx;
  g.ny = c->lv[l].ny;
  g.h = c->lv[l].h;
  g.m = c->lv[l].m.as<double>();
  g.mstride = c->lv[l].mstride;
  g.rho = c->has_rho ? c->lv[l].rho.as<double>() : nullptr;
  g.dc = (c->has_rho && c->dim == 2) ? c->lv[l].dc.as<double>() : nullptr;
  if (l == 0) g.px = c->fine_px;
  return g;
}

// the slot stride of level l's vectors (the finest level's rows may be pitched)
size_t level_stride(const hz_ctx* c, int l) {
  return (l == 0 && c->fine_px > 0) ? (size_t)c->lv[0].nz * c->fine_px : c->lv[l].n();
}

// Local Fourier analysis of damped Jacobi on h^2 M: for a mode with Laplacian
// symbol l the error factor is 1 - w (l - s q)/(2 dim - s q), s = beta1 - j
// beta2, q = (kh)^2; over the high-frequency modes l runs through
// [2, 4 dim], and the modulus of this affine function of l peaks at an end.
double smoothing_factor(double kh, double b1, double b2, double w, int dim) {
  const std::complex<double> s(b1, -b2);
  const double q = kh * kh;
  const std::complex<double> den = 2.0 * dim - s * q;
  auto amp = [&](double l) { return std::abs(1.0 - w * (l - s * q) / den); };
  return std::max(amp(2.0), amp(4.0 * dim));
}

const double kWeights[] = {0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2};
constexpr int kKhSamples = 65;

}  // namespace

namespace hz {

// Level hierarchy. An axis of n nodes halves to ceil(n / 2): coarse node J
// sits on fine node 2J; with an even n the last fine node has no coarse
// partner and is interpolated from the last coarse node alone.
int coarse_n(int n) { return (n + 1) / 2; }

// Largest level count a grid allows: halve while every axis keeps >= 3 nodes.
int grid_max_levels(int dim, int nz, int nx) {
  int L = 1;
  while (L < kMaxLevels && nx >= 5 && (dim == 1 || nz >= 5)) {
    nx = coarse_n(nx);
    if (dim == 2) nz = coarse_n(nz);
    ++L;
  }
  return L;
}

// Levels of a default plan: halve while the coarsest level has more than
// kCoarseTarget unknowns (a deeper hierarchy with a small dense coarse solve
// took fewer or equal BiCGSTAB iterations than stopping at ~1300 unknowns on
// the layered 401 x 801 model at 3-12 Hz, and each iteration costs less).
constexpr long kCoarseTarget = 512;

int grid_default_levels(int dim, int nz, int nx) {
  int L = 1;
  while (L < kMaxLevels && (long)nx * nz > kCoarseTarget && nx >= 5 && (dim == 1 || nz >= 5)) {
    nx = coarse_n(nx);
    if (dim == 2) nz = coarse_n(nz);
    ++L;
  }
  return L;
}

// The same two counts on a 3D grid (every axis halves).
int grid_max_levels3(int nz, int ny, int nx) {
  int L = 1;
  while (L < kMaxLevels && nz >= 5 && ny >= 5 && nx >= 5) {
    nz = coarse_n(nz);
    ny = coarse_n(ny);
    nx = coarse_n(nx);
    ++L;
  }
  return L;
}

int grid_default_levels3(int nz, int ny, int nx) {
  int L = 1;
  while (L < kMaxLevels && (long)nz * ny * nx > kCoarseTarget && nz >= 5 && ny >= 5 && nx >= 5) {
    nz = coarse_n(nz);
    ny = coarse_n(ny);
    nx = coarse_n(nx);
    ++L;
  }
  return L;
}

}  // namespace hz

namespace {

// Whether the V-cycle of L levels solves its coarsest level exactly at this
// frequency (as setup_freqs decides), and how many unknowns that level has.
bool coarse_is_exact(const hz_solve_opts* o, int L, double hc, double mmin, double omega) {
  if (o->precond != HZ_PRECOND_MG) return false;
  if (L == 1 || o->coarse == HZ_COARSE_EXACT) return true;
  return o->coarse == HZ_COARSE_AUTO && !(omega * hc * mmin >= 2.5);
}

size_t coarsest_nodes(int dim, int nz, int ny, int nx, int L) {
  for (int l = 1; l < L; ++l) {
    nx = coarse_n(nx);
    if (dim >= 2) nz = coarse_n(nz);
    if (dim == 3) ny = coarse_n(ny);
  }
  return (size_t)nx * (dim >= 2 ? nz : 1) * (dim == 3 ? ny : 1);
}

// The level count and per-level Jacobi weights for one frequency; refuses
// (HZ_ERR_SHAPE) a plan whose coarsest level is solved exactly and holds
// more than kCoarseMax unknowns.
int plan_grid(int dim, int nz, int ny, int nx, int maxlev, int deflev, double h, double mmin, double mmax,
              const hz_solve_opts* o, double omega, int* levels, double* w) {
  int L = o->levels > 0 ? o->levels : deflev;
  if (L > maxlev) return HZ_ERR_SHAPE;
  if (coarse_is_exact(o, L, h * ldexp(1.0, L - 1), mmin, omega) &&
      coarsest_nodes(dim, nz, ny, nx, L) > (size_t)kCoarseMax)
    return HZ_ERR_SHAPE;
  *levels = L;
  for (int l = 0; l < L - 1; ++l) {
    if (o->jacobi_w_level) {
      w[l] = o->jacobi_w_level[l];
      continue;
    }
    const double hl = h * ldexp(1.0, l);
    const double lo = omega * hl * mmin, hi = omega * hl * mmax;
    double chosen = -1.0, best = -1.0, best_mu = 0.0;
    for (double cand : kWeights) {
      if (cand > o->jacobi_w + 1e-12) continue;
      double worst = 0.0;
      for (int i = 0; i < kKhSamples; ++i) {
        const double kh = lo + (hi - lo) * i / (double)(kKhSamples - 1);
        worst = std::max(worst, smoothing_factor(kh, o->beta1, o->beta2, cand, dim));
      }
      if (worst <= 1.0) {
        chosen = cand;
        break;
      }
      if (best < 0.0 || worst < best_mu) {
        best = cand;
        best_mu = worst;
      }
    }
    w[l] = chosen > 0.0 ? chosen : (best > 0.0 ? best : o->jacobi_w);
  }
  return HZ_OK;
}

int default_levels_of(const hz_ctx* c) {
  return c->dim == 3 ? grid_default_levels3(c->nz, c->ny, c->nx) : grid_default_levels(c->dim, c->nz, c->nx);
}

int make_plan(const hz_ctx* c, const hz_solve_opts* o, double omega, int* levels, double* w) {
  return plan_grid(c->dim, c->nz, c->ny, c->nx, c->maxlev, default_levels_of(c), c->h, c->mmin, c->mmax, o, omega,
                   levels, w);
}

int check_opts(hz_ctx* c, const hz_solve_opts* o) {
  if (!(o->tol > 0.0) || !isfinite(o->tol)) return fail(c, HZ_ERR_ARG, "tol must be positive");
  if (o->maxit < 1) return fail(c, HZ_ERR_ARG, "maxit must be >= 1");
  if (o->krylov != HZ_BICGSTAB && o->krylov != HZ_GMRES) return fail(c, HZ_ERR_ARG, "unknown krylov method");
  if (o->krylov == HZ_GMRES && (o->gmres_m < 1 || o->gmres_m > 200))
    return fail(c, HZ_ERR_ARG, "gmres_m must be in [1, 200]");
  if (o->precond < HZ_PRECOND_MG || o->precond > HZ_PRECOND_NONE) return fail(c, HZ_ERR_ARG, "unknown preconditioner");
  if (o->precond != HZ_PRECOND_NONE) {
    if (!(o->beta2 > 0.0) || !isfinite(o->beta1) || !isfinite(o->beta2))
      return fail(c, HZ_ERR_ARG, "the shift needs beta2 > 0 and finite beta1");
  }
  if (o->precond == HZ_PRECOND_MG) {
    if (o->nu1 < 1 || o->nu2 < 0 || o->nu1 > 16 || o->nu2 > 16)
      return fail(c, HZ_ERR_ARG, "need 1 <= nu1 <= 16 and 0 <= nu2 <= 16");
    if (!(o->jacobi_w > 0.0 && o->jacobi_w <= 1.0)) return fail(c, HZ_ERR_ARG, "jacobi_w must be in (0, 1]");
    if (o->levels < 0) return fail(c, HZ_ERR_ARG, "levels must be >= 0");
    if (o->levels > c->maxlev)
      return fail(c, HZ_ERR_SHAPE, "the grid allows at most %d levels", c->maxlev);
    if (o->jacobi_w_level) {
      const int L = o->levels > 0 ? o->levels : default_levels_of(c);
      for (int l = 0; l < L - 1; ++l)
        if (!(o->jacobi_w_level[l] > 0.0 && o->jacobi_w_level[l] <= 1.0))
          return fail(c, HZ_ERR_ARG, "jacobi_w_level[%d] must be in (0, 1]", l);
    }
  }
  if (o->chunk_rows < 0 || (o->chunk_rows & 1) || o->chunk_rows > (1 << 16))
    return fail(c, HZ_ERR_ARG, "chunk_rows must be 0 or an even number up to 65536");
  if (o->autotune != 0 && o->autotune != 1) return fail(c, HZ_ERR_ARG, "autotune must be 0 or 1");
  if (o->graphs != 0 && o->graphs != 1) return fail(c, HZ_ERR_ARG, "graphs must be 0 or 1");
  if (o->restart_at < 0) return fail(c, HZ_ERR_ARG, "restart_at must be >= 0");
  if (o->plain != 0 && o->plain != 1) return fail(c, HZ_ERR_ARG, "plain must be 0 or 1");
  if (o->coarse < HZ_COARSE_AUTO || o->coarse > HZ_COARSE_JACOBI) return fail(c, HZ_ERR_ARG, "unknown coarse solve");
  if (o->coarse_sweeps < 1 || o->coarse_sweeps > 64) return fail(c, HZ_ERR_ARG, "coarse_sweeps must be in [1, 64]");
  if (o->precond == HZ_PRECOND_EXACT) {
    if (c->dim != 1) return fail(c, HZ_ERR_ARG, "the exact preconditioner is the 1D tridiagonal solve");
    const size_t lds = (size_t)4 * c->nx * sizeof(double2);
    if (c->nx > kPcrMax || lds > c->max_lds)
      return fail(c, HZ_ERR_ARG, "1D grid of %d nodes is too long for the exact tridiagonal solve", c->nx);
  }
  return HZ_OK;
}

// ---------------------------------------------------------------- workspace
int ensure_workspace(hz_ctx* c, int nslots, int levels) {
  const size_t n0 = fine_nodes(c->dim, c->lv[0].nz, c->lv[0].ny, c->lv[0].nx);
  size_t total = 0;
  total += (size_t)kNumFine * nslots * n0 * sizeof(double2);
  for (int l = 1; l < levels; ++l) total += (size_t)kNumLevelVec * nslots * c->lv[l].n() * sizeof(double2);
  if (c->budget && total > c->budget)
    return fail(c, HZ_ERR_NOMEM, "workspace of %zu bytes exceeds the budget of %zu", total, c->budget);
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < kNumFine; ++k) HZ_ALLOC(c, c->fine[k], (size_t)nslots * n0 * sizeof(double2));
  for (int l = 1; l < levels; ++l)
    for (int k = 0; k < kNumLevelVec; ++k)
      HZ_ALLOC(c, c->lev[l][k], (size_t)nslots * c->lv[l].n() * sizeof(double2));
  // reduction scratch: enough tiles for any kernel on the fine grid
  const Tiles t = grid_tiles(c->lv[0].rows(), c->lv[0].nx, c->dim);
  const int tiles = std::max({t.per_slot, reduce_tiles(c->lv[0].rows(), c->lv[0].nx, c->dim), vec_tiles(n0)});
  if (nslots > c->slot_cap || tiles > c->partial_tiles) {
    const int cap = std::max(nslots, c->slot_cap);
    HZ_ALLOC(c, c->partials, (size_t)cap * tiles * kPartialWidth * sizeof(double));
    HZ_ALLOC(c, c->slots, (size_t)cap * sizeof(Slot));
    HZ_ALLOC(c, c->rh_idx, (size_t)cap * kShadowMax * sizeof(int));
    HZ_ALLOC(c, c->rh_val, (size_t)cap * kShadowMax * sizeof(double2));
    HZ_ALLOC(c, c->active, (size_t)cap * sizeof(int));
    HZ_ALLOC(c, c->nactive, sizeof(int) * 4);
    HZ_ALLOC(c, c->resid, (size_t)cap * 2 * sizeof(double));
    c->slot_cap = cap;
    c->partial_tiles = tiles;
  }
  c->ws_slots = nslots;
  c->ws_levels = levels;
  return HZ_OK;
}

Reduce reducer(const hz_ctx* c) {
  Reduce r;
  r.partials = c->partials.as<double>();
  r.max_tiles = c->partial_tiles;
  return r;
}

Batch batch_of(const hz_ctx* c) {
  Batch b;
  b.active = c->active.as<int>();
  b.nactive = c->nactive.as<int>();
  b.slots = c->slots.as<Slot>();
  b.ft = c->freqtab.as<FreqTab>();
  b.fstart = c->fstart.as<int>();
  b.rh_idx = c->rh_idx.as<int>();
  b.rh_val = c->rh_val.as<double2>();
  return b;
}

// The list 0..n-1 of every slot and its per-frequency ranges.
int reset_list(hz_ctx* c, int nslots, int nrhs) {
  const int nfreq = nslots / nrhs;
  std::vector<int> act(nslots), fs(nfreq + 1);
  for (int i = 0; i < nslots; ++i) act[i] = i;
  for (int f = 0; f <= nfreq; ++f) fs[f] = f * nrhs;
  HZ_ALLOC(c, c->fstart, (size_t)(nfreq + 1) * sizeof(int));
  HZ_HIP(c, hipMemcpyAsync(c->active.p, act.data(), nslots * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(c->nactive.p, &nslots, sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(c->fstart.p, fs.data(), (nfreq + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  c->cur_nfreq = nfreq;
  c->cur_nrhs = nrhs;
  return HZ_OK;
}

// Upload slot records (all active, frequency = slot / nrhs) and the full list.
int reset_slots(hz_ctx* c, int nslots, int nrhs) {
  std::vector<Slot> s(nslots);
  for (int i = 0; i < nslots; ++i) {
    memset(&s[i], 0, sizeof(Slot));
    s[i].status = kActive;
    s[i].freq = i / nrhs;
    s[i].rh_nnz = -1;
  }
  HZ_HIP(c, hipMemcpyAsync(c->slots.p, s.data(), nslots * sizeof(Slot), hipMemcpyHostToDevice, c->stream));
  return reset_list(c, nslots, nrhs);
}

// Build the per-frequency table; invert the coarsest M when the V-cycle needs it.
int setup_freqs(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha,
                int levels, const std::vector<std::vector<double>>& wj) {
  std::vector<FreqTab> ft(nfreq);
  for (int f = 0; f < nfreq; ++f) {
    memset(&ft[f], 0, sizeof(FreqTab));
    ft[f].omega = 2.0 * M_PI * freq_hz[f];
    ft[f].sB_re = 1.0;
    ft[f].sB_im = -alpha;
    ft[f].sM_re = o->beta1;
    ft[f].sM_im = -o->beta2;
    for (int l = 0; l < levels - 1 && l < (int)wj[f].size(); ++l) ft[f].wj[l] = wj[f][l];
  }
  HZ_ALLOC(c, c->freqtab, (size_t)nfreq * sizeof(FreqTab));
  if (o->precond == HZ_PRECOND_MG && levels > 1) {
    size_t tot = 0;
    for (int l = 0; l < levels - 1; ++l) tot += c->lv[l].n();
    HZ_ALLOC(c, c->winv, tot * nfreq * sizeof(double2));
    double2* wp = c->winv.as<double2>();
    for (int f = 0; f < nfreq; ++f) {
      for (int l = 0; l < levels - 1; ++l) {
        HZ_HIP(c, launch_winv(c->dim, grid_of(c, l), ft[f].omega, ft[f].sM_re, ft[f].sM_im, ft[f].wj[l], wp,
                              c->stream));
        ft[f].winv[l] = wp;
        wp += c->lv[l].n();
      }
    }
  }
  const bool need_coarse = o->precond == HZ_PRECOND_MG;
  c->any_coarse_jacobi = false;
  if (need_coarse && levels > 1) {
    // damped Jacobi on the coarsest level converges for every mode once its
    // smallest kh reaches 2.5 (local Fourier analysis of the shifted Laplacian)
    const double hc = c->lv[levels - 1].h;
    for (int f = 0; f < nfreq; ++f) {
      const bool jac = o->coarse == HZ_COARSE_JACOBI ||
                       (o->coarse == HZ_COARSE_AUTO && ft[f].omega * hc * c->mmin >= 2.5);
      ft[f].coarse_jacobi = jac ? 1 : 0;
      c->any_coarse_jacobi = c->any_coarse_jacobi || jac;
    }
  }
  // the dense inverse is needed unless every frequency smooths its coarsest level
  bool need_inverse = false;
  for (int f = 0; f < nfreq; ++f) need_inverse = need_inverse || !(levels > 1 && ft[f].coarse_jacobi);
  if (need_coarse && need_inverse) {
    const int cl = levels - 1;
    const size_t nc = c->lv[cl].n();
    if (nc > (size_t)kCoarseMax)
      return fail(c, HZ_ERR_SHAPE, "coarsest level has %zu unknowns (limit %d); allow more levels", nc, kCoarseMax);
    std::vector<double> key;
    key.push_back(c->model_version);
    key.push_back(levels);
    key.push_back(o->beta1);
    key.push_back(o->beta2);
    for (int f = 0; f < nfreq; ++f) key.push_back(ft[f].omega);
    if (key != c->cinv_key || !c->cinv_base) {
      const size_t bytes = nc * nc * nfreq * sizeof(double2);
      if (c->budget && bytes * 2 > c->budget)
        return fail(c, HZ_ERR_NOMEM, "coarse inverses need %zu bytes", bytes * 2);
      HZ_ALLOC(c, c->cinv_a, bytes);
      HZ_ALLOC(c, c->cinv_b, bytes);
      HZ_HIP(c, hipMemcpyAsync(c->freqtab.p, ft.data(), nfreq * sizeof(FreqTab), hipMemcpyHostToDevice, c->stream));
      HZ_HIP(c, launch_assemble_dense(c->dim, grid_of(c, cl), nfreq, c->freqtab.as<FreqTab>(),
                                      c->cinv_a.as<double2>(), c->stream));
      double2* src = c->cinv_a.as<double2>();
      double2* dst = c->cinv_b.as<double2>();
      for (size_t k = 0; k < nc; ++k) {
        HZ_HIP(c, launch_gj_step((int)nc, nfreq, (int)k, src, dst, c->stream));
        std::swap(src, dst);
      }
      c->cinv_base = src;
      c->cinv_key = key;
    }
    for (int f = 0; f < nfreq; ++f) ft[f].cinv = c->cinv_base + (size_t)f * nc * nc;
  }
  HZ_HIP(c, hipMemcpyAsync(c->freqtab.p, ft.data(), nfreq * sizeof(FreqTab), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

// Event pair around one launch of the timed kernel class (no-op otherwise).
hipEvent_t take_event(hz_ctx* c) {
  if (!c->tpool.empty()) {
    hipEvent_t e = c->tpool.back();
    c->tpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <class F>
hipError_t timed(hz_ctx* c, int cls, F&& launch) {
  if (cls < 0 || !(c->timing_mask & (1u << cls)) || c->noalloc) return launch();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, c->stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, c->stream);
  c->tpairs.push_back({a, b, cls});
  return e;
}

// Fold recorded pairs into the totals (the stream must have been synchronised).
void fold_timing(hz_ctx* c) {
  for (auto& pr : c->tpairs) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pr.a, pr.b) == hipSuccess) {
      c->t_ms[pr.cls] += ms;
      c->t_launches[pr.cls] += 1;
    }
    c->tpool.push_back(pr.a);
    c->tpool.push_back(pr.b);
  }
  c->tpairs.clear();
}

// ---------------------------------------------------------------- V-cycle
struct Cycle {
  int levels, nu1, nu2, precond;
  int autotune, chunk_rows;  // launch shape of the fused kernels (opts.autotune, opts.chunk_rows)
  int coarse_sweeps;         // > 0: some frequency smooths its coarsest level with this many sweeps
  int plain;                 // opts.plain: one kernel per step, dense r^, host readback every iteration
  int unfused;               // no fused V-cycle kernels (opts.plain, or a density on a 1D or 3D grid)
};

// ---------------------------------------------------------------- launch-shape tuning
// The wave-streaming fused kernels take the number of grid rows each
// wavefront marches over. Short chunks give more wavefronts (better for small
// levels and small batches), long ones re-read fewer halo rows. The tuner
// times every candidate once per (kernel, level grid, batch-size octave) on
// the real operands, at the first launch with that key, and keeps the
// fastest. The kernels are pure (they never write what they read), so the
// trial launches leave the same result as one launch.
constexpr int kChunkCandidates[] = {2, 4, 8, 16, 32, 64, 128};
constexpr double kCoarseJacobiW = 0.8;  // weight of the coarsest-level sweeps (HZ_COARSE_JACOBI)
constexpr int kChunkDefault = 32;

int octave(int cap) {
  int b = 0;
  while (b < 30 && (2 << b) <= cap) ++b;
  return b;
}

// Shapes tuned by any context of the process, per device (contexts created
// later, such as the server's engines, start from them).
std::mutex g_tuned_mu;
std::map<std::array<int, 5>, int> g_tuned;

template <class F>
hipError_t tuned_launch(hz_ctx* c, const Cycle& cy, int kind, const Grid& g, int cap, F launch) {
  if (cy.chunk_rows > 0) return launch(cy.chunk_rows);
  const std::array<int, 4> key{kind, g.nz, g.nx, octave(cap)};
  auto it = c->tuned_chunk.find(key);
  if (it != c->tuned_chunk.end()) return launch(it->second);
  const std::array<int, 5> gkey{c->device, kind, g.nz, g.nx, octave(cap)};
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto gt = g_tuned.find(gkey);
    if (gt != g_tuned.end()) {
      c->tuned_chunk[key] = gt->second;
      return launch(gt->second);
    }
  }
  if (!cy.autotune || c->noalloc) return launch(kChunkDefault);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int pick = kChunkDefault;
  float best = 0.0f;
  bool have = false;
  for (int ch : kChunkCandidates) {
    if (e != hipSuccess) break;
    if (ch / 2 >= g.nz && ch != kChunkCandidates[0]) break;  // one chunk already covers the grid
    if ((e = launch(ch)) != hipSuccess) break;               // warm-up
    if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
    if ((e = launch(ch)) != hipSuccess) break;
    if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    if (!have || ms < best) {
      best = ms;
      pick = ch;
      have = true;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  c->tuned_chunk[key] = pick;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned.emplace(gkey, pick);
  }
  return launch(pick);
}

// How the finest level's right-hand side is formed: read (mode 0), or the
// BiCGSTAB vector p = a + beta (b - omega c) (mode 1) or s = a - alpha b
// (mode 2), stored to `out` by the kernel that forms it. 2D only: modes 4
// and 5 take p^ in c and form its product with B themselves, p = a + beta
// (b - omega B c) (a where beta = 0) and s = a - alpha B c.
struct FineRhs {
  int mode;
  const double2* a;
  const double2* b;
  const double2* c;
  double2* out;
};

bool fused_pre(const Cycle& cy) {
  return cy.precond == HZ_PRECOND_MG && cy.levels >= 2 && cy.nu1 == 2 && !cy.unfused;
}

// out = V b on the finest grid for the slots of the active list. With rhs
// (fused path only) the finest right-hand side is formed by the first kernel.
hipError_t precond_apply(hz_ctx* c, const Cycle& cy, int cap, const double2* b0, double2* out,
                         const FineRhs* rhs = nullptr) {
  const Batch bt = batch_of(c);
  const int dim = c->dim;
  hipStream_t st = c->stream;
  const size_t n0 = c->lv[0].n();
  if (cy.precond == HZ_PRECOND_NONE) return launch_copy(bt, cap, n0, b0, out, n0, st);
  if (cy.precond == HZ_PRECOND_EXACT) return launch_pcr(grid_of(c, 0), bt, cap, b0, out, n0, st);
  const int L = cy.levels;
  if (L == 1) return launch_coarse_solve((int)n0, c->cur_nfreq, c->cur_nrhs, bt, b0, out, n0, st);
  hipError_t e;
  if (rhs) b0 = rhs->out;
  // 2D V(2,2): the levels from the first one with at most kSmallNodes nodes
  // down to the coarsest are walked by two kernels (one workgroup per
  // right-hand side) instead of a launch per level and step
  // (the first level small enough whose vectors also fit the workgroup's LDS)
  int l0 = L;
  SmallLevels sl;
  memset(&sl, 0, sizeof sl);
  if (dim == 2 && cy.nu1 == 2 && cy.nu2 == 2 && !cy.unfused && L >= 3)
    for (int lf = 1; lf < L - 1 && l0 == L; ++lf) {
      if (c->lv[lf].n() > (size_t)kSmallNodes) continue;
      sl.l0 = lf;
      sl.L = L;
      sl.coarse_sweeps = cy.coarse_sweeps;
      sl.coarse_w = kCoarseJacobiW;
      for (int l = lf; l < L; ++l) {
        sl.g[l] = grid_of(c, l);
        sl.b[l] = c->lev[l][kLb].as<double2>();
        sl.u[l] = c->lev[l][kLu].as<double2>();
        sl.x[l] = c->lev[l][kLx].as<double2>();
        sl.y[l] = c->lev[l][kLy].as<double2>();
        sl.n[l] = c->lv[l].n();
      }
      if (small_levels_lds(sl) <= c->max_lds) l0 = lf;
    }
  const int ldesc = std::min(L - 1, l0);  // levels with per-level launches
  // descend
  const double2* bl = b0;
  double2* cur[kMaxLevels];
  for (int l = 0; l < ldesc; ++l) {
    const Grid g = grid_of(c, l);
    const size_t nl = level_stride(c, l);
    double2* X = l == 0 ? c->fine[kT1].as<double2>() : c->lev[l][kLx].as<double2>();
    double2* Y = l == 0 ? c->fine[kT2].as<double2>() : c->lev[l][kLy].as<double2>();
    double2* u = nullptr;
    double2* bc = c->lev[l + 1][kLb].as<double2>();
    // the fused post-smoothing kernel forms the pre-smoothed iterate again
    const bool post_fused = dim == 2 && cy.nu1 == 2 && cy.nu2 >= 2 && !cy.unfused;
    if (cy.nu1 == 2 && dim == 2 && !cy.unfused) {
      // both pre-sweeps, the residual and its restriction in one pass
      const FineRhs plain{0, bl, nullptr, nullptr, nullptr};
      const FineRhs& fr = (l == 0 && rhs) ? *rhs : plain;
      const Grid gc = grid_of(c, l + 1);
      const size_t nc = c->lv[l + 1].n();
      const int cls =
          l > 0 ? HZ_KERNEL_LEVELS : (fr.mode == 2 || fr.mode == 5 ? HZ_KERNEL_PRESMOOTH_S : HZ_KERNEL_PRESMOOTH);
      if ((e = timed(c, cls, [&] {
             return tuned_launch(c, cy, fr.mode, g, cap, [&](int ch) {
               return launch_pre2r(g, gc, l, fr.mode, bt, cap, fr.a, fr.b, fr.c, fr.out, post_fused ? nullptr : X,
                                   bc, nl, nc, ch, st);
             });
           })) != hipSuccess)
        return e;
      cur[l] = X;
      bl = bc;
      continue;
    }
    if (cy.nu1 == 2 && dim == 3 && !cy.unfused) {
      // both pre-sweeps from zero in one marching pass
      if ((e = timed(c, l == 0 ? HZ_KERNEL_SMOOTH : HZ_KERNEL_LEVELS, [&] {
             return launch_march3(g, l, bt, cap, true, bl, nullptr, X, nl, st);
           })) != hipSuccess)
        return e;
      u = X;
    } else if (cy.nu1 == 2 && dim == 1 && !cy.unfused) {
      const FineRhs plain{0, bl, nullptr, nullptr, nullptr};
      const FineRhs& fr = (l == 0 && rhs) ? *rhs : plain;
      if ((e = timed(c, l == 0 ? HZ_KERNEL_PRESMOOTH : HZ_KERNEL_LEVELS, [&] {
             return launch_pre2(dim, g, l, fr.mode, bt, cap, fr.a, fr.b, fr.c, fr.out, X, nl, st);
           })) != hipSuccess)
        return e;
      u = X;
    } else {
      for (int k = 0; k < cy.nu1; ++k) {
        double2* dst = (u == X) ? Y : X;
        const int cls = l > 0 ? HZ_KERNEL_LEVELS : (u ? HZ_KERNEL_SMOOTH : -2);
        if ((e = timed(c, cls, [&] { return launch_smooth(dim, g, l, 0.0, bt, cap, bl, u, dst, nl, st); })) !=
            hipSuccess)
          return e;
        u = dst;
      }
    }
    cur[l] = u;
    // the level's other smoothing buffer holds the residual where the restriction stores it first
    double2* spare = (u == X) ? Y : X;
    if ((e = timed(c, l == 0 ? HZ_KERNEL_RESTRICT : HZ_KERNEL_LEVELS, [&] {
           return launch_restrict_via(dim, g, grid_of(c, l + 1), bt, cap, bl, u, spare, bc, nl, c->lv[l + 1].n(),
                                      st);
         })) != hipSuccess)
      return e;
    bl = bc;
  }
  if (l0 < L - 1) {
    const int cl = L - 1;
    if ((e = timed(c, HZ_KERNEL_LEVELS, [&] { return launch_vdown(sl, bt, cap, st); })) != hipSuccess) return e;
    // the exact coarse solve (frequencies that smooth their coarsest level were done in the descent)
    if ((e = timed(c, HZ_KERNEL_COARSE, [&] {
           return launch_coarse_solve((int)c->lv[cl].n(), c->cur_nfreq, c->cur_nrhs, bt, c->lev[cl][kLb].as<double2>(),
                                      c->lev[cl][kLu].as<double2>(), c->lv[cl].n(), st);
         })) != hipSuccess)
      return e;
    if ((e = timed(c, HZ_KERNEL_LEVELS, [&] { return launch_vup(sl, bt, cap, st); })) != hipSuccess) return e;
  } else {
    // coarsest
    const int cl = L - 1;
    if ((e = timed(c, HZ_KERNEL_COARSE, [&] {
           return launch_coarse_solve((int)c->lv[cl].n(), c->cur_nfreq, c->cur_nrhs, bt, c->lev[cl][kLb].as<double2>(),
                                      c->lev[cl][kLu].as<double2>(), c->lv[cl].n(), st);
         })) != hipSuccess)
      return e;
    // frequencies whose coarsest level is smoothed (the exact solve skipped them)
    if (cy.coarse_sweeps > 0 && (e = timed(c, HZ_KERNEL_LEVELS, [&] {
                                   return launch_coarse_jacobi(dim, grid_of(c, cl), cl, kCoarseJacobiW,
                                                               cy.coarse_sweeps, bt, cap, c->lev[cl][kLb].as<double2>(),
                                                               c->lev[cl][kLx].as<double2>(),
                                                               c->lev[cl][kLu].as<double2>(), c->lv[cl].n(), st);
                                 })) != hipSuccess)
      return e;
  }
  // ascend
  for (int l = ldesc - 1; l >= 0; --l) {
    const Grid g = grid_of(c, l);
    const Grid gc = grid_of(c, l + 1);
    const size_t nl = level_stride(c, l);
    double2* X = l == 0 ? c->fine[kT1].as<double2>() : c->lev[l][kLx].as<double2>();
    double2* Y = l == 0 ? c->fine[kT2].as<double2>() : c->lev[l][kLy].as<double2>();
    double2* R = l == 0 ? out : c->lev[l][kLu].as<double2>();
    const double2* bll = l == 0 ? b0 : c->lev[l][kLb].as<double2>();
    const double2* ec = c->lev[l + 1][kLu].as<double2>();
    double2* u = cur[l];
    if (cy.nu2 == 0) {
      if ((e = timed(c, l == 0 ? HZ_KERNEL_PROLONG : HZ_KERNEL_LEVELS, [&] {
             return launch_prolong(dim, g, gc, bt, cap, ec, u, R, nl, c->lv[l + 1].n(), st);
           })) != hipSuccess)
        return e;
      continue;
    }
    // prolongation fused with the first post-sweep (2D, and 3D with a constant density: with
    // the first two)
    const bool post3 = dim == 3 && !g.rho && cy.nu2 >= 2 && !cy.unfused;
    const int fused = ((dim == 2 && cy.nu1 == 2 && cy.nu2 >= 2 && !cy.unfused) || post3) ? 2 : 1;
    double2* dst = (cy.nu2 == fused) ? R : ((u == X) ? Y : X);
    if ((e = timed(c, l == 0 ? HZ_KERNEL_PROLONG : HZ_KERNEL_LEVELS, [&] {
           if (post3) return launch_post3(g, gc, l, bt, cap, bll, u, ec, dst, nl, c->lv[l + 1].n(), st);
           if (fused == 2)
             return tuned_launch(c, cy, 3, g, cap, [&](int ch) {
               return launch_post2(g, gc, l, bt, cap, ec, bll, dst, nl, c->lv[l + 1].n(), ch, st);
             });
           if (dim == 3 && !g.rho && !cy.unfused)
             // 3D: the marching sweep forms u + P e where it reads the iterate
             return launch_march3(g, l, bt, cap, false, bll, u, dst, nl, st, &gc, ec, c->lv[l + 1].n());
           if (dim == 3) {
             // 3D with a density: u += P e in place (the pre-smoothed iterate is not needed
             // after), then a sweep
             hipError_t e3 = launch_prolong(dim, g, gc, bt, cap, ec, u, u, nl, c->lv[l + 1].n(), st);
             if (e3 == hipSuccess) e3 = launch_smooth(dim, g, l, 0.0, bt, cap, bll, u, dst, nl, st);
             return e3;
           }
           return launch_prolong_smooth(dim, g, gc, l, bt, cap, ec, bll, u, dst, nl, c->lv[l + 1].n(), st);
         })) != hipSuccess)
      return e;
    u = dst;
    for (int k = fused; k < cy.nu2; ++k) {
      double2* d2 = (k == cy.nu2 - 1) ? R : ((u == X) ? Y : X);
      if ((e = timed(c, l == 0 ? HZ_KERNEL_SMOOTH : HZ_KERNEL_LEVELS, [&] {
             return launch_smooth(dim, g, l, 0.0, bt, cap, bll, u, d2, nl, st);
           })) != hipSuccess)
        return e;
      u = d2;
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- BiCGSTAB driver
// The vectors and flags of a BiCGSTAB run over the context's slots, and one
// iteration of it for the first entries of the active list.
struct BicgIter {
  hz_ctx* c;
  const hz_solve_opts* o;
  Cycle cy;
  size_t n0;
  Batch bt;
  Reduce rd;
  Grid g0;
  double2 *r, *rh, *pbuf[2], *p, *v, *s, *t, *x;
  double2 *phr[2], *shr[2], *ph, *sh;
  bool identity, fused, vfree, defer;
  bool dense_rh = false;  // some active slot's r^ is a dense vector
  // pitched: the finest-level vectors and the iterate have rows of pitch
  // c->fine_px (the caller's b and x stay [nz][nx])
  bool pitched = false;
  double2* xp = nullptr;
  int vt, gt;

  // allow_pitch: the solve may lay the finest level out with pitched rows
  // (hz_solve; the serving engine keeps [nz][nx])
  BicgIter(hz_ctx* cc, const hz_solve_opts* oo, const Cycle& cyy, double2* xx, bool allow_pitch = false)
      : c(cc), o(oo), cy(cyy), x(xx) {
    fused = fused_pre(cy) && c->dim != 3;
    vfree = fused && c->dim == 2;
    // every finest-level kernel of the fused 2D path with V(2,2) reads the
    // pitch; other shapes sweep the finest level with kernels that do not
    pitched = allow_pitch && vfree && cy.nu2 == 2 && fine_pitch(c->lv[0].nx) != c->lv[0].nx;
    c->fine_px = pitched ? fine_pitch(c->lv[0].nx) : 0;
    n0 = level_stride(c, 0);
    bt = batch_of(c);
    rd = reducer(c);
    g0 = grid_of(c, 0);
    r = c->fine[kR].as<double2>();
    rh = c->fine[kRh].as<double2>();
    pbuf[0] = c->fine[kP].as<double2>();
    pbuf[1] = c->fine[kP2].as<double2>();
    p = pbuf[0];
    v = c->fine[kV].as<double2>();
    s = c->fine[kS].as<double2>();
    t = c->fine[kT].as<double2>();
    if (pitched) {  // v and t are not stored on this path: v's buffer holds the iterate
      xp = v;
      x = xp;
      v = nullptr;
      t = nullptr;
    }
    identity = cy.precond == HZ_PRECOND_NONE;
    // 2D with the fused pre-smoothing kernel: v = B p^ is never stored. The
    // pre-smoothing kernels form it from p^ (the last iteration's p^ for the p
    // update, the current one for s), and sigma = <r^, B p^> is formed at the
    // nodes of r^'s sparse list. Slots whose r^ is dense (a right-hand side
    // with many nonzeros, or after a restart) take sigma from an operator pass
    // that stores nothing, launched while any active slot needs it (vfree).
    // The iterate is advanced every second iteration: p^ and s^ of iteration
    // 2k (ring 0) stay in their buffers while 2k+1 (ring 1) writes the others,
    // and ring 1's update adds both terms (one read and write of x instead of
    // two). Without a preconditioner s^ = s is overwritten at once, so x is
    // advanced every iteration.
    defer = !identity && !cy.plain;
    phr[0] = c->fine[kPh].as<double2>();
    phr[1] = c->fine[kPh2].as<double2>();
    shr[0] = identity ? s : c->fine[kSh].as<double2>();
    shr[1] = identity ? s : c->fine[kSh2].as<double2>();
    ph = phr[0];
    sh = shr[0];
    vt = vec_tiles(c->lv[0].n());  // tiles of the init and restart passes (and of the flat update)
    gt = reduce_tiles(c->lv[0].rows(), c->lv[0].nx, c->dim);  // tiles of the operator-apply kernels
  }

  // Start the slots of the list `lb` (cap entries): x = 0, r = r^ = b, the
  // initial scalars and (unless plain) the sparse lists of r^ for the slots
  // slot0 .. slot0 + nlist - 1.
  hipError_t start(const Batch& lb, int cap, const double2* b, int slot0, int nlist) {
    hipStream_t st = c->stream;
    const size_t nd = c->lv[0].n();  // the caller's b: [nz][nx] per slot
    // (pitched: r, r^, p and x take the nodes at their pitched places; the padding is never read)
    hipError_t e = launch_bicg_init(nd, lb, cap, rd, b, x, r, rh, p, v, n0, st, nd, c->lv[0].nx, c->fine_px);
    if (e == hipSuccess) e = launch_bicg_fin(kFinInit, vt, lb, cap, rd, o->tol, o->maxit, nullptr, n0, st);
    // the plain path keeps every r^ dense (rh_nnz = -1 in the slot records); the
    // list holds node indices iz * nx + ix
    if (e == hipSuccess && !cy.plain)
      e = launch_rh_sparse(nd, nlist, lb, b, c->rh_idx.as<int>(), c->rh_val.as<double2>(), nd, st, slot0);
    return e;
  }

  // The pitched iterate into the caller's x ([nz][nx] per slot).
  hipError_t finish(double2* xout, int nslots) {
    if (!pitched) return hipSuccess;
    const int nz = c->lv[0].nz, nx = c->lv[0].nx;
    return launch_repitch(nslots, nz, nx, xp, c->fine_px, n0, xout, nx, c->lv[0].n(), c->stream);
  }

  // One BiCGSTAB iteration for the first `capx` entries of the active list,
  // issued on stream `sx` (every launch of the path reads c->stream).
  hipError_t issue(int capx, hipStream_t sx, int ring) {
    const hipStream_t saved = c->stream;
    c->stream = sx;
    hipError_t e = hipSuccess;
    const int rg = defer ? ring : -1;
    if (!identity) {
      ph = phr[ring];
      sh = shr[ring];
    }
    // p_new = r + beta (p_old - omega v) into the other p buffer, then ph = V p_new
    double2* pn = (p == pbuf[0]) ? pbuf[1] : pbuf[0];
    do {
      if (vfree) {  // the last iteration's p^ is in the other ring buffer
        const FineRhs fr{4, r, p, phr[ring ^ 1], pn};
        if ((e = precond_apply(c, cy, capx, nullptr, ph, &fr)) != hipSuccess) break;
      } else if (fused) {
        const FineRhs fr{1, r, p, v, pn};
        if ((e = precond_apply(c, cy, capx, nullptr, ph, &fr)) != hipSuccess) break;
      } else {
        if ((e = launch_bicg_p(n0, bt, capx, r, p, v, pn, n0, sx)) != hipSuccess) break;
        if (!identity && (e = precond_apply(c, cy, capx, pn, ph)) != hipSuccess) break;
      }
      p = pn;
      if (identity) ph = p;
      if (vfree) {
        if (dense_rh && (e = timed(c, HZ_KERNEL_APPLY, [&] {
                           return launch_bicg_apply_sigma(c->dim, g0, bt, capx, rd, ph, rh, nullptr, n0, sx);
                         })) != hipSuccess)
          break;
        if ((e = launch_bicg_fin(kFinSigmaB, gt, bt, capx, rd, o->tol, o->maxit, ph, n0, sx, -1, 0, &g0)) !=
            hipSuccess)
          break;
      } else {
        if ((e = timed(c, HZ_KERNEL_APPLY, [&] {
               return launch_bicg_apply_sigma(c->dim, g0, bt, capx, rd, ph, rh, v, n0, sx);
             })) != hipSuccess)
          break;
        if ((e = launch_bicg_fin(kFinSigma, gt, bt, capx, rd, o->tol, o->maxit, v, n0, sx)) != hipSuccess) break;
      }
      if (vfree) {
        const FineRhs fr{5, r, nullptr, ph, s};
        if ((e = precond_apply(c, cy, capx, nullptr, sh, &fr)) != hipSuccess) break;
      } else if (fused) {
        const FineRhs fr{2, r, v, nullptr, s};
        if ((e = precond_apply(c, cy, capx, nullptr, sh, &fr)) != hipSuccess) break;
      } else {
        if ((e = launch_bicg_s(n0, bt, capx, r, v, s, n0, sx)) != hipSuccess) break;
        if (!identity && (e = precond_apply(c, cy, capx, s, sh)) != hipSuccess) break;
      }
      // 2D fused path: t = B s^ is not stored; the update forms it again from s^
      if ((e = timed(c, HZ_KERNEL_APPLY_S, [&] {
             return launch_bicg_apply_omega(c->dim, g0, bt, capx, rd, sh, s, vfree ? nullptr : t, n0, sx);
           })) != hipSuccess)
        break;
      if ((e = launch_bicg_fin(kFinOmega, gt, bt, capx, rd, o->tol, o->maxit, nullptr, n0, sx)) != hipSuccess)
        break;
      if ((e = timed(c, HZ_KERNEL_UPDATE, [&] {
             return vfree ? launch_bicg_xr_t(g0, bt, capx, rd, x, ph, sh, s, r, rh, n0, sx, rg, phr[0], shr[0])
                          : launch_bicg_xr(n0, bt, capx, rd, x, ph, sh, s, t, r, rh, n0, sx, rg, phr[0], shr[0]);
           })) != hipSuccess)
        break;
      // (the fused path gathers r at the list's nodes through the grid: its rows may be pitched)
      e = launch_bicg_fin(kFinStep, vfree ? gt : vt, bt, capx, rd, o->tol, o->maxit, r, n0, sx, rg,
                          o->restart_at, vfree ? &g0 : nullptr);
    } while (false);
    c->stream = saved;
    return e;
  }

  // The one restart after a breakdown for the slots waiting for it (their
  // pending iterate terms added first).
  hipError_t restart(int nslots) {
    hipStream_t st = c->stream;
    hipError_t e = hipSuccess;
    if (defer) e = launch_bicg_flush(n0, nslots, bt, 1, x, phr[0], shr[0], n0, st);
    if (e == hipSuccess)  // current p buffer
      e = launch_bicg_restart(c->lv[0].n(), nslots, bt, rd, r, rh, p, v, n0, st, c->lv[0].nx, c->fine_px);
    if (e == hipSuccess) e = launch_bicg_fin(kFinRestart, vt, bt, nslots, rd, o->tol, o->maxit, nullptr, n0, st);
    dense_rh = true;  // r^ = r for the restarted slots
    return e;
  }
};

int run_bicgstab(hz_ctx* c, const hz_solve_opts* o, const Cycle& cy, int nslots,
                 const double2* b, double2* x) {
  BicgIter it(c, o, cy, x, true);
  struct PitchReset {  // the pitched layout ends with this solve, on every return
    hz_ctx* c;
    ~PitchReset() { c->fine_px = 0; }
  } pitch_reset{c};
  const Batch bt = it.bt;
  const size_t n0 = it.n0;
  hipStream_t st = c->stream;

  long long seq = 0;                 // units issued
  long long restart_seq = -1;        // last unit that was a restart
  std::deque<std::pair<long long, int>> pending;  // (unit, ring slot)
  int ring_next = 0;
  auto close_unit = [&]() -> int {
    const int k = ring_next;
    ring_next = (ring_next + 1) % kRing;
    HZ_HIP(c, launch_compact(nslots, c->cur_nrhs, c->cur_nfreq, bt.slots, c->active.as<int>(),
                             c->nactive.as<int>(), c->fstart.as<int>(), c->ring_dev + k, 0, st));
    HZ_HIP(c, hipEventRecord(c->ev[k], st));
    pending.emplace_back(seq++, k);
    return HZ_OK;
  };

  int rc;
  HZ_HIP(c, it.start(bt, nslots, b, 0, nslots));
  if ((rc = close_unit()) != HZ_OK) return rc;
  if (it.vfree) {  // whether the first iterations need the dense sigma pass
    const int k = pending.back().second;
    HZ_HIP(c, hipEventSynchronize(c->ev[k]));
    it.dense_rh = c->ring_host[k].ndense > 0;
  }

  int cap = nslots;
  long long iters_issued = 0;
  const long long guard = 2LL * (o->maxit + 2) + 16;
  bool done = false;
  auto issue_iteration = [&](int capx, hipStream_t sx, int ring) { return it.issue(capx, sx, ring); };

  // HIP graphs: two iterations (the p buffers swap twice, so a pair starts
  // and ends on the same buffer) captured once per batch-size bucket (the
  // active count rounded up to a power of two; launches past the active
  // list exit at once) and whether the dense sigma pass is in, and replayed. The first pair of a bucket runs
  // eagerly, which also runs the launch-shape trials, so nothing that
  // synchronises is captured. Kernel timing needs per-launch events, so
  // timed solves run eagerly.
  const bool use_graphs = o->graphs && c->timing_mask == 0 && !cy.plain && !c->noalloc;
  // summaries in flight before the host waits: the plain path reads every
  // iteration's back before it issues the next
  const int lag = cy.plain ? 0 : kLag;
  struct GraphSet {  // instantiated graphs of this solve, destroyed once the stream is idle
    hipStream_t st;
    std::map<int, hipGraphExec_t> m;
    ~GraphSet() {
      if (m.empty()) return;
      (void)hipStreamSynchronize(st);
      for (auto& kv : m) (void)hipGraphExecDestroy(kv.second);
    }
  } gset{st, {}};
  std::map<int, hipGraphExec_t>& graphs = gset.m;
  std::map<int, int> eager_pairs;
  auto bucket = [&](int n) {
    int b = 1;
    while (b < n) b <<= 1;
    return std::min(b, nslots);
  };
  auto issue_pair_graph = [&](int capx) -> int {
    const int cb = bucket(capx);
    const int key = 2 * cb + (it.dense_rh ? 1 : 0);
    auto it = graphs.find(key);
    if (it == graphs.end() && eager_pairs[key] == 0) {
      eager_pairs[key] = 1;
      HZ_HIP(c, issue_iteration(cb, st, 0));
      HZ_HIP(c, issue_iteration(cb, st, 1));
      return HZ_OK;
    }
    if (it == graphs.end()) {
      if (!c->graph_stream) HZ_HIP(c, hipStreamCreateWithFlags(&c->graph_stream, hipStreamNonBlocking));
      hipGraph_t gr = nullptr;
      HZ_HIP(c, hipStreamBeginCapture(c->graph_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = issue_iteration(cb, c->graph_stream, 0);
      if (e == hipSuccess) e = issue_iteration(cb, c->graph_stream, 1);
      const hipError_t e2 = hipStreamEndCapture(c->graph_stream, &gr);
      if (e == hipSuccess) e = e2;
      hipGraphExec_t ex = nullptr;
      if (e == hipSuccess) e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      if (gr) (void)hipGraphDestroy(gr);
      if (e != hipSuccess)
        return fail(c, HZ_ERR_DEVICE, "capturing the iteration graph failed: %s", hipGetErrorString(e));
      it = graphs.emplace(key, ex).first;
    }
    HZ_HIP(c, hipGraphLaunch(it->second, st));
    return HZ_OK;
  };

  while (!done) {
    while (!pending.empty() && ((int)pending.size() > lag || cap == 0)) {
      const auto [useq, k] = pending.front();
      pending.pop_front();
      HZ_HIP(c, hipEventSynchronize(c->ev[k]));
      const Summary sm = c->ring_host[k];
      const bool stale = restart_seq > useq;
      if (!stale) {
        cap = std::min(cap, sm.nactive);
        if (sm.nrestart == 0) it.dense_rh = sm.ndense > 0;
        if (sm.nrestart > 0) {
          HZ_HIP(c, it.restart(nslots));
          restart_seq = seq;
          if ((rc = close_unit()) != HZ_OK) return rc;
          cap = nslots;
        } else if (sm.nactive == 0) {
          done = true;
          break;
        }
      }
    }
    if (done) break;
    if (cap == 0) {
      if (pending.empty()) break;
      continue;
    }
    if (iters_issued >= guard) break;
    if (use_graphs) {
      if ((rc = issue_pair_graph(cap)) != HZ_OK) return rc;
      iters_issued += 2;
    } else {
      HZ_HIP(c, issue_iteration(cap, st, (int)(iters_issued & 1)));
      ++iters_issued;
    }
    if ((rc = close_unit()) != HZ_OK) return rc;
  }
  // terms of slots that stopped after a ring-0 update
  if (it.defer) HZ_HIP(c, launch_bicg_flush(n0, nslots, bt, 0, it.x, it.phr[0], it.shr[0], n0, st));
  HZ_HIP(c, it.finish(x, nslots));
  HZ_HIP(c, hipStreamSynchronize(st));
  fold_timing(c);
  return HZ_OK;
}

// ---------------------------------------------------------------- GMRES(m) driver
// All slots run one restart cycle in lockstep: Arnoldi step j is launched for
// the slots still in phase 0; a slot whose residual estimate meets tol (or
// that reaches maxit or step m) moves to phase 1 and waits. When none is left
// in phase 0 the cycle ends for all: y = H^-1 g, x += M^-1 (V y), and the
// true residual starts the next cycle or finishes the slot.
int run_gmres(hz_ctx* c, const hz_solve_opts* o, const Cycle& cy, int nslots, const double2* b,
              double2* x) {
  const int m = o->gmres_m;
  const size_t n0 = c->lv[0].n();
  const size_t vstride = (size_t)nslots * n0;
  const int tiles = std::max(vec_tiles(n0), gm_dot_tiles(n0));
  const size_t vbytes = (size_t)(m + 1) * vstride * sizeof(double2);
  if (c->budget && vbytes > c->budget)
    return fail(c, HZ_ERR_NOMEM, "GMRES basis of %zu bytes exceeds the budget", vbytes);
  HZ_ALLOC(c, c->gm_V, vbytes);
  const size_t m1 = (size_t)m + 1;
  const size_t nH = (size_t)nslots * m1 * m, ng = (size_t)nslots * m1, nsn = (size_t)nslots * m;
  const size_t nhc = (size_t)nslots * 2 * m1;
  const int width = 4 * (m + 1) + 4;
  HZ_ALLOC(c, c->gm_small, (2 * nH + ng + nsn + nsn + nhc) * sizeof(double2) + nsn * sizeof(double));
  HZ_ALLOC(c, c->gm_part, (size_t)nslots * tiles * width * sizeof(double));
  Gmres gm;
  double2* base = c->gm_small.as<double2>();
  gm.H = base;
  gm.Hu = gm.H + nH;
  gm.g = gm.Hu + nH;
  gm.sn = gm.g + ng;
  gm.y = gm.sn + nsn;
  gm.hc = gm.y + nsn;
  gm.cs = reinterpret_cast<double*>(gm.hc + nhc);
  gm.partials = c->gm_part.as<double>();
  gm.m = m;
  gm.max_tiles = tiles;
  gm.width = width;

  const Batch bt = batch_of(c);
  const Reduce rd = reducer(c);
  const Grid g0 = grid_of(c, 0);
  hipStream_t st = c->stream;
  const bool identity = cy.precond == HZ_PRECOND_NONE;
  double2* V = c->gm_V.as<double2>();
  double2* z = c->fine[kPh].as<double2>();
  double2* t = c->fine[kT].as<double2>();

  std::deque<std::pair<long long, int>> pending;
  long long seq = 0;
  int ring_next = 0;
  auto close_unit = [&](int phase) -> int {
    const int k = ring_next;
    ring_next = (ring_next + 1) % kRing;
    HZ_HIP(c, launch_compact(nslots, c->cur_nrhs, c->cur_nfreq, bt.slots, c->active.as<int>(),
                             c->nactive.as<int>(), c->fstart.as<int>(), c->ring_dev + k, phase, st));
    HZ_HIP(c, hipEventRecord(c->ev[k], st));
    pending.emplace_back(seq++, k);
    return HZ_OK;
  };
  auto drain = [&](Summary* last) -> int {
    while (!pending.empty()) {
      const int k = pending.front().second;
      pending.pop_front();
      HZ_HIP(c, hipEventSynchronize(c->ev[k]));
      *last = c->ring_host[k];
    }
    return HZ_OK;
  };

  int rc;
  Summary sm{};
  HZ_HIP(c, launch_gm_residual(c->dim, g0, bt, nslots, rd, gm, 1, o->tol, o->maxit, b, x, V, n0, st));
  if ((rc = close_unit(0)) != HZ_OK) return rc;
  if ((rc = drain(&sm)) != HZ_OK) return rc;
  int cap = sm.nactive;
  if (cap > 0) HZ_HIP(c, launch_gm_scale(n0, bt, cap, V, n0, st));
  const long long guard = (long long)o->maxit + 2;
  long long cycles = 0;
  while (cap > 0 && cycles++ <= guard) {
    // step j applies the operator to u_j (V_j, not yet normalised) into
    // V_{j+1}; the step's kernels then finish v_j in place and overwrite
    // V_{j+1} with u_{j+1}. Column j - 1 is decided at step j, column m - 1 by
    // the finishing pass.
    int j = 0;
    for (; j < m && cap > 0; ++j) {
      const double2* uj = V + (size_t)j * vstride;
      double2* w = V + (size_t)(j + 1) * vstride;
      const double2* zin = uj;
      if (!identity) {
        HZ_HIP(c, precond_apply(c, cy, cap, uj, z));
        zin = z;
      }
      HZ_HIP(c, timed(c, HZ_KERNEL_APPLY, [&] { return launch_apply(c->dim, g0, 0, 0, bt, cap, zin, w, n0, st); }));
      HZ_HIP(c, timed(c, HZ_KERNEL_UPDATE, [&] {
               return launch_gm_step(n0, bt, cap, gm, j, 0, o->tol, o->maxit, V, vstride, w, n0, st);
             }));
      if ((rc = close_unit(0)) != HZ_OK) return rc;
      while ((int)pending.size() > (cy.plain ? 0 : kLag)) {
        const int k = pending.front().second;
        pending.pop_front();
        HZ_HIP(c, hipEventSynchronize(c->ev[k]));
        cap = std::min(cap, c->ring_host[k].nactive);
      }
    }
    if (j == m && cap > 0) {
      HZ_HIP(c, timed(c, HZ_KERNEL_UPDATE, [&] {
               return launch_gm_step(n0, bt, cap, gm, m, 1, o->tol, o->maxit, V, vstride, nullptr, n0, st);
             }));
      if ((rc = close_unit(0)) != HZ_OK) return rc;
    }
    if ((rc = drain(&sm)) != HZ_OK) return rc;
    // cycle end for every slot waiting in phase 1
    if ((rc = close_unit(1)) != HZ_OK) return rc;
    if ((rc = drain(&sm)) != HZ_OK) return rc;
    const int n1 = sm.nactive;
    if (n1 == 0) break;
    HZ_HIP(c, launch_gm_solve(bt, n1, gm, st));
    HZ_HIP(c, launch_gm_combine(n0, bt, n1, gm, V, vstride, t, n0, st));
    const double2* upd = t;
    if (!identity) {
      HZ_HIP(c, precond_apply(c, cy, n1, t, z));
      upd = z;
    }
    HZ_HIP(c, launch_axpy1(n0, bt, n1, upd, x, n0, st));
    HZ_HIP(c, launch_gm_residual(c->dim, g0, bt, n1, rd, gm, 0, o->tol, o->maxit, b, x, V, n0, st));
    if ((rc = close_unit(0)) != HZ_OK) return rc;
    if ((rc = drain(&sm)) != HZ_OK) return rc;
    cap = sm.nactive;
    if (cap > 0) HZ_HIP(c, launch_gm_scale(n0, bt, cap, V, n0, st));
  }
  HZ_HIP(c, hipStreamSynchronize(st));
  fold_timing(c);
  return HZ_OK;
}

// Final statuses and true residuals for every slot.
int collect_info(hz_ctx* c, int nslots, const double2* b, const double2* x, hz_rhs_info* info,
                 int* any_fail) {
  int rc = reset_list(c, nslots, c->cur_nrhs);
  if (rc) return rc;
  HZ_HIP(c, launch_true_residual(c->dim, grid_of(c, 0), batch_of(c), nslots, reducer(c), b, x,
                                 c->resid.as<double>(), c->lv[0].n(), c->stream));
  std::vector<Slot> s(nslots);
  std::vector<double> res(2 * nslots);
  HZ_HIP(c, hipMemcpyAsync(s.data(), c->slots.p, nslots * sizeof(Slot), hipMemcpyDeviceToHost, c->stream));
  HZ_HIP(c, hipMemcpyAsync(res.data(), c->resid.p, 2 * nslots * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  *any_fail = 0;
  for (int i = 0; i < nslots; ++i) {
    int stt = s[i].status;
    if (stt == kActive) stt = kMaxit;
    if (stt == kRestart) stt = kBreakdown;
    if (stt != kConverged) *any_fail = 1;
    if (info) {
      info[i].status = stt;
      info[i].iters = s[i].iters;
      info[i].relres = res[2 * i + 1] > 0.0 ? sqrt(res[2 * i]) / sqrt(res[2 * i + 1]) : 0.0;
      info[i].seconds = c->wall_khz > 0.0 ? (double)(s[i].t1 - s[i].t0) / (c->wall_khz * 1e3) : 0.0;
    }
  }
  return HZ_OK;
}

int require_model(hz_ctx* c) {
  if (!c) return HZ_ERR_ARG;
  if (c->dim == 0) return fail(c, HZ_ERR_STATE, "no model set");
  return HZ_OK;
}

int setup_debug_batch(hz_ctx* c, int nrhs, double freq_hz, double alpha, double beta1, double beta2,
                      const double* wj, int nwj) {
  if (nrhs < 1) return fail(c, HZ_ERR_ARG, "nrhs must be >= 1");
  if (!(freq_hz > 0.0) || !isfinite(freq_hz)) return fail(c, HZ_ERR_ARG, "frequency must be positive");
  int rc = ensure_workspace(c, nrhs, std::max(c->ws_levels, 1));
  if (rc) return rc;
  FreqTab ft;
  memset(&ft, 0, sizeof ft);
  ft.omega = 2.0 * M_PI * freq_hz;
  ft.sB_re = 1.0;
  ft.sB_im = -alpha;
  ft.sM_re = beta1;
  ft.sM_im = -beta2;
  for (int l = 0; l < nwj && l < kMaxLevels; ++l) ft.wj[l] = wj[l];
  HZ_ALLOC(c, c->freqtab, sizeof(FreqTab));
  HZ_HIP(c, hipMemcpyAsync(c->freqtab.p, &ft, sizeof ft, hipMemcpyHostToDevice, c->stream));
  return reset_slots(c, nrhs, nrhs);
}

}  // namespace

// ================================================================ C ABI
extern "C" {

void hz_default_opts(hz_solve_opts* o) {
  if (!o) return;
  o->krylov = HZ_BICGSTAB;
  o->gmres_m = 30;
  o->tol = 1e-8;
  o->maxit = 10000;
  o->precond = HZ_PRECOND_MG;
  o->beta1 = 1.0;
  o->beta2 = 0.5;
  o->levels = 0;
  o->nu1 = 2;
  o->nu2 = 2;
  o->jacobi_w = 0.8;
  o->jacobi_w_level = nullptr;
  o->autotune = 1;
  o->chunk_rows = 0;
  o->coarse = HZ_COARSE_AUTO;
  o->coarse_sweeps = 2;
  o->graphs = 0;
  o->restart_at = 0;
  o->plain = 0;
}

int hz_create(hz_ctx** out, const hz_ctx_opts* o) {
  if (!out || !o) return HZ_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev) return HZ_ERR_ARG;
  hz_ctx* c = new hz_ctx();
  c->device = o->device;
  c->stream = static_cast<hipStream_t>(o->hip_stream);
  c->budget = o->workspace_budget_bytes;
  if (hipSetDevice(c->device) != hipSuccess) {
    delete c;
    return HZ_ERR_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    delete c;
    return HZ_ERR_DEVICE;
  }
  c->max_lds = prop.sharedMemPerBlock;
  int wkhz = 0;
  if (hipDeviceGetAttribute(&wkhz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess) c->wall_khz = wkhz;
  void* ring = nullptr;
  if (hipHostMalloc(&ring, kRing * sizeof(Summary), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete c;
    return HZ_ERR_NOMEM;
  }
  c->ring_host = static_cast<Summary*>(ring);
  memset(ring, 0, kRing * sizeof(Summary));
  void* dptr = nullptr;
  if (hipHostGetDevicePointer(&dptr, ring, 0) != hipSuccess) {
    (void)hipHostFree(ring);
    delete c;
    return HZ_ERR_DEVICE;
  }
  c->ring_dev = static_cast<Summary*>(dptr);
  // the allocation-free solve's array on this device (device current); a
  // failed lookup is reported by hz_solve_noalloc, the other calls do not need it
  c->scratch_status = scratch_setup(c->device);
  for (int k = 0; k < kRing; ++k) {
    if (hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming) != hipSuccess) {
      hz_destroy(c);
      return HZ_ERR_DEVICE;
    }
  }
  *out = c;
  return HZ_OK;
}

void hz_destroy(hz_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (int k = 0; k < kRing; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
  fold_timing(c);
  for (hipEvent_t e : c->tpool) (void)hipEventDestroy(e);
  if (c->ring_host) (void)hipHostFree(c->ring_host);
  if (c->graph_stream) (void)hipStreamDestroy(c->graph_stream);
  delete c;
}

namespace {
// The model of any dimension (ny = 1 below 3D); arguments checked by the callers.
int set_model_impl(hz_ctx* c, int dim, int nz, int ny, int nx, double h, const double* m_dev) {
  HZ_HIP(c, hipSetDevice(c->device));
  const size_t n = (size_t)nz * ny * nx;
  HZ_ALLOC(c, c->lv[0].m, n * sizeof(double));
  HZ_HIP(c, hipMemcpyAsync(c->lv[0].m.p, m_dev, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  DevBuf chk;
  HZ_ALLOC(c, chk, 4 * sizeof(double));
  HZ_HIP(c, launch_check_model(n, c->lv[0].m.as<double>(), chk.as<double>(), c->stream));
  double out3[3];
  HZ_HIP(c, hipMemcpyAsync(out3, chk.p, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  if (out3[2] > 0.0) {
    c->dim = 0;
    return fail(c, HZ_ERR_ARG, "slowness has %.0f entries that are not finite and positive", out3[2]);
  }
  c->dim = dim;
  c->nz = nz;
  c->ny = ny;
  c->nx = nx;
  c->h = h;
  c->mmin = c->m_lo = out3[0];
  c->mmax = c->m_hi = out3[1];
  c->has_rho = 0;  // a new model starts at constant density
  c->lv[0].nz = nz;
  c->lv[0].ny = ny;
  c->lv[0].nx = nx;
  c->lv[0].h = h;
  int L = 1;
  while (L < kMaxLevels) {
    const LevelInfo& f = c->lv[L - 1];
    if (f.nx < 5 || (dim >= 2 && f.nz < 5) || (dim == 3 && f.ny < 5)) break;
    LevelInfo& cl = c->lv[L];
    cl.nx = coarse_n(f.nx);
    cl.nz = dim == 1 ? 1 : coarse_n(f.nz);
    cl.ny = dim == 3 ? coarse_n(f.ny) : 1;
    cl.h = 2.0 * f.h;
    HZ_ALLOC(c, cl.m, cl.n() * sizeof(double));
    HZ_HIP(c, launch_inject(grid_of(c, L - 1), dim, cl.m.as<double>(), c->stream));
    ++L;
  }
  c->maxlev = L;
  c->model_version += 1;
  c->cinv_key.clear();
  c->cinv_base = nullptr;
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

}  // namespace

int hz_set_model(hz_ctx* c, int dim, int nz, int nx, double h, const double* m_dev) {
  if (!c) return HZ_ERR_ARG;
  if (!m_dev) return fail(c, HZ_ERR_ARG, "m_dev is NULL");
  if (dim != 1 && dim != 2) return fail(c, HZ_ERR_ARG, "dim must be 1 or 2 (3D grids: hz_set_model_3d)");
  if (dim == 1 && (nz != 1 || nx < 3)) return fail(c, HZ_ERR_ARG, "1D needs nz = 1 and nx >= 3");
  if (dim == 2 && (nz < 3 || nx < 3)) return fail(c, HZ_ERR_ARG, "2D needs nz, nx >= 3");
  if ((size_t)nz * nx > (size_t)1 << 30) return fail(c, HZ_ERR_ARG, "grid too large");
  if (!(h > 0.0) || !isfinite(h)) return fail(c, HZ_ERR_ARG, "h must be positive");
  return set_model_impl(c, dim, nz, 1, nx, h, m_dev);
}

int hz_set_density(hz_ctx* c, const double* rho_dev) {
  if (!c) return HZ_ERR_ARG;
  if (c->dim < 1 || c->dim > 3) return fail(c, HZ_ERR_ARG, "a density needs a model set first");
  HZ_HIP(c, hipSetDevice(c->device));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  if (!rho_dev) {
    c->has_rho = 0;
    c->mmin = c->m_lo;
    c->mmax = c->m_hi;
  } else {
    const size_t n = c->lv[0].n();
    HZ_ALLOC(c, c->lv[0].rho, n * sizeof(double));
    HZ_HIP(c, hipMemcpyAsync(c->lv[0].rho.p, rho_dev, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    DevBuf chk;
    HZ_ALLOC(c, chk, 4 * sizeof(double));
    HZ_HIP(c, launch_check_density(n, c->lv[0].m.as<double>(), c->lv[0].rho.as<double>(), chk.as<double>(),
                                   c->stream));
    double out3[3];
    HZ_HIP(c, hipMemcpyAsync(out3, chk.p, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HZ_HIP(c, hipStreamSynchronize(c->stream));
    if (out3[2] > 0.0) {
      c->has_rho = 0;
      c->mmin = c->m_lo;
      c->mmax = c->m_hi;
      return fail(c, HZ_ERR_ARG, "density has %.0f entries that are not finite and positive", out3[2]);
    }
    // injected to the coarse levels like the slowness
    for (int l = 1; l < c->maxlev; ++l) {
      HZ_ALLOC(c, c->lv[l].rho, c->lv[l].n() * sizeof(double));
      Grid gf = grid_of(c, l - 1);
      gf.m = c->lv[l - 1].rho.as<double>();
      HZ_HIP(c, launch_inject(gf, c->dim, c->lv[l].rho.as<double>(), c->stream));
    }
    // 2D: every level's coupling table for the fused kernels
    if (c->dim == 2)
      for (int l = 0; l < c->maxlev; ++l) {
        HZ_ALLOC(c, c->lv[l].dc, 3 * c->lv[l].n() * sizeof(double));
        Grid gl = grid_of(c, l);
        gl.rho = c->lv[l].rho.as<double>();
        HZ_HIP(c, launch_density_coef(gl, c->lv[l].dc.as<double>(), c->stream));
      }
    HZ_HIP(c, hipStreamSynchronize(c->stream));
    c->has_rho = 1;
    c->mmin = out3[0];
    c->mmax = out3[1];
  }
  c->model_version += 1;
  c->cinv_key.clear();
  c->cinv_base = nullptr;
  return HZ_OK;
}

int hz_set_model_3d(hz_ctx* c, int nz, int ny, int nx, double h, const double* m_dev) {
  if (!c) return HZ_ERR_ARG;
  if (!m_dev) return fail(c, HZ_ERR_ARG, "m_dev is NULL");
  if (nz < 3 || ny < 3 || nx < 3) return fail(c, HZ_ERR_ARG, "3D needs nz, ny, nx >= 3");
  if ((size_t)nz * ny * nx > (size_t)1 << 30) return fail(c, HZ_ERR_ARG, "grid too large");
  if (!(h > 0.0) || !isfinite(h)) return fail(c, HZ_ERR_ARG, "h must be positive");
  return set_model_impl(c, 3, nz, ny, nx, h, m_dev);
}

namespace {
// b_dev[s] = amp_s / h^dim at node nodes[s] (flat index), zero elsewhere
int set_points(hz_ctx* c, const std::vector<int>& nodes, const hz_c128* amp, hz_c128* b_dev) {
  const int nsrc = (int)nodes.size();
  HZ_HIP(c, hipSetDevice(c->device));
  HZ_ALLOC(c, c->scratch_int, (size_t)nsrc * sizeof(int));
  HZ_HIP(c, hipMemcpyAsync(c->scratch_int.p, nodes.data(), nsrc * sizeof(int), hipMemcpyHostToDevice, c->stream));
  const double2* ampd = nullptr;
  if (amp) {
    HZ_ALLOC(c, c->scratch_c, (size_t)nsrc * sizeof(double2));
    HZ_HIP(c, hipMemcpyAsync(c->scratch_c.p, amp, nsrc * sizeof(double2), hipMemcpyHostToDevice, c->stream));
    ampd = c->scratch_c.as<double2>();
  }
  const double scale = c->dim == 1 ? 1.0 / c->h : (c->dim == 2 ? 1.0 / (c->h * c->h) : 1.0 / std::pow(c->h, 3.0));
  HZ_HIP(c, launch_point_rhs(c->lv[0].n(), nsrc, c->scratch_int.as<int>(), ampd, scale,
                             reinterpret_cast<double2*>(b_dev), c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}
}  // namespace

int hz_point_rhs(hz_ctx* c, int nsrc, const int* iz, const int* ix, const hz_c128* amp,
                 hz_c128* b_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  if (c->dim == 3) return fail(c, HZ_ERR_ARG, "the model is 3D: use hz_point_rhs_3d");
  if (nsrc < 1 || !iz || !ix || !b_dev) return fail(c, HZ_ERR_ARG, "bad point-source arguments");
  std::vector<int> nodes(nsrc);
  for (int s = 0; s < nsrc; ++s) {
    if (iz[s] < 0 || iz[s] >= c->nz || ix[s] < 0 || ix[s] >= c->nx)
      return fail(c, HZ_ERR_ARG, "source %d at (%d, %d) is outside the grid", s, iz[s], ix[s]);
    nodes[s] = iz[s] * c->nx + ix[s];
  }
  return set_points(c, nodes, amp, b_dev);
}

int hz_point_rhs_3d(hz_ctx* c, int nsrc, const int* iz, const int* iy, const int* ix, const hz_c128* amp,
                    hz_c128* b_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  if (c->dim != 3) return fail(c, HZ_ERR_ARG, "the model is not 3D: use hz_point_rhs");
  if (nsrc < 1 || !iz || !iy || !ix || !b_dev) return fail(c, HZ_ERR_ARG, "bad point-source arguments");
  std::vector<int> nodes(nsrc);
  for (int s = 0; s < nsrc; ++s) {
    if (iz[s] < 0 || iz[s] >= c->nz || iy[s] < 0 || iy[s] >= c->ny || ix[s] < 0 || ix[s] >= c->nx)
      return fail(c, HZ_ERR_ARG, "source %d at (%d, %d, %d) is outside the grid", s, iz[s], iy[s], ix[s]);
    nodes[s] = (iz[s] * c->ny + iy[s]) * c->nx + ix[s];
  }
  return set_points(c, nodes, amp, b_dev);
}

int hz_plan(const hz_ctx* c, const hz_solve_opts* o, double freq_hz, int* levels, double* w) {
  if (!c || !levels || !w) return HZ_ERR_ARG;
  if (c->dim == 0) return HZ_ERR_STATE;
  hz_solve_opts d;
  if (!o) {
    hz_default_opts(&d);
    o = &d;
  }
  if (!(freq_hz > 0.0)) return HZ_ERR_ARG;
  for (int l = 0; l < HZ_MAX_LEVELS; ++l) w[l] = 0.0;
  return make_plan(c, o, 2.0 * M_PI * freq_hz, levels, w);
}

int hz_plan_grid(int dim, int nz, int nx, double h, double m_min, double m_max,
                 const hz_solve_opts* o, double freq_hz, int* levels, double* w) {
  if (!levels || !w) return HZ_ERR_ARG;
  if ((dim != 1 && dim != 2) || nx < 3 || (dim == 1 ? nz != 1 : nz < 3)) return HZ_ERR_ARG;
  if (!(h > 0.0) || !(m_min > 0.0) || !(m_max >= m_min) || !(freq_hz > 0.0)) return HZ_ERR_ARG;
  hz_solve_opts d;
  if (!o) {
    hz_default_opts(&d);
    o = &d;
  }
  for (int l = 0; l < HZ_MAX_LEVELS; ++l) w[l] = 0.0;
  return plan_grid(dim, nz, 1, nx, grid_max_levels(dim, nz, nx), grid_default_levels(dim, nz, nx), h, m_min, m_max,
                   o, 2.0 * M_PI * freq_hz, levels, w);
}

namespace {
int solve_impl(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nrhs,
               const hz_c128* b_dev, hz_c128* u_dev, hz_rhs_info* info) {
  int rc = require_model(c);
  if (rc) return rc;
  hz_solve_opts d;
  if (!o) {
    hz_default_opts(&d);
    o = &d;
  }
  if (nfreq < 1 || nrhs < 0 || !freq_hz) return fail(c, HZ_ERR_ARG, "bad solve arguments");
  if (!(alpha >= 0.0) || !isfinite(alpha)) return fail(c, HZ_ERR_ARG, "alpha must be >= 0");
  for (int f = 0; f < nfreq; ++f)
    if (!(freq_hz[f] > 0.0) || !isfinite(freq_hz[f])) return fail(c, HZ_ERR_ARG, "frequency %d must be positive", f);
  if ((rc = check_opts(c, o)) != HZ_OK) return rc;
  if (nrhs == 0) return HZ_OK;  // an empty batch: nothing to solve
  if (!b_dev || !u_dev) return fail(c, HZ_ERR_ARG, "bad solve arguments");
  if ((long long)nfreq * nrhs > (1 << 20)) return fail(c, HZ_ERR_ARG, "too many right-hand sides");
  const int nslots = nfreq * nrhs;
  const size_t n0 = c->lv[0].n();
  {
    const char* bb = reinterpret_cast<const char*>(b_dev);
    const char* uu = reinterpret_cast<const char*>(u_dev);
    const size_t bytes = (size_t)nslots * n0 * sizeof(double2);
    if (bb < uu + bytes && uu < bb + bytes) return fail(c, HZ_ERR_ARG, "b_dev and u_dev overlap");
  }
  HZ_HIP(c, hipSetDevice(c->device));
  int levels = 1;
  std::vector<std::vector<double>> wj(nfreq, std::vector<double>(kMaxLevels, 0.0));
  if (o->precond == HZ_PRECOND_MG) {
    for (int f = 0; f < nfreq; ++f) {
      int L = 0;
      if ((rc = make_plan(c, o, 2.0 * M_PI * freq_hz[f], &L, wj[f].data())) != HZ_OK)
        return fail(c, rc,
                    "cannot plan the V-cycle: more levels than the grid allows, or an exactly solved "
                    "coarsest level above %d unknowns",
                    kCoarseMax);
      levels = L;
    }
  }
  if ((rc = ensure_workspace(c, nslots, levels)) != HZ_OK) return rc;
  if ((rc = setup_freqs(c, o, nfreq, freq_hz, alpha, levels, wj)) != HZ_OK) return rc;
  if ((rc = reset_slots(c, nslots, nrhs)) != HZ_OK) return rc;
  const Cycle cy{levels, o->nu1, o->nu2, o->precond, o->autotune, o->chunk_rows,
                 c->any_coarse_jacobi ? o->coarse_sweeps : 0, o->plain, o->plain || (c->has_rho && c->dim != 2)};
  const double2* b = reinterpret_cast<const double2*>(b_dev);
  double2* x = reinterpret_cast<double2*>(u_dev);
  if (o->krylov == HZ_BICGSTAB) {
    rc = run_bicgstab(c, o, cy, nslots, b, x);
  } else {
    rc = run_gmres(c, o, cy, nslots, b, x);
  }
  if (rc) return rc;
  int any_fail = 0;
  if ((rc = collect_info(c, nslots, b, x, info, &any_fail)) != HZ_OK) return rc;
  return any_fail ? HZ_WARN_NOCONV : HZ_OK;
}
}  // namespace

int hz_solve(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha,
             int nrhs, const hz_c128* b_dev, hz_c128* u_dev, hz_rhs_info* info) {
  return solve_impl(c, o, nfreq, freq_hz, alpha, nrhs, b_dev, u_dev, info);
}

namespace {

// Moves the context's solver workspace aside (and its cached coarse
// inverses, workspace sizes and slot capacity) so that the solve finds
// every buffer empty and takes it from the arena; puts everything back on
// destruction, after the stream has drained.
struct WorkspaceStash {
  hz_ctx* c;
  std::vector<DevBuf*> bufs;
  struct Saved {
    void* p;
    size_t bytes;
    bool borrowed;
  };
  std::vector<Saved> saved;
  int ws_slots, ws_levels, slot_cap, partial_tiles;
  std::vector<double> cinv_key;
  const double2* cinv_base;
  explicit WorkspaceStash(hz_ctx* cc) : c(cc) {
    for (auto& b : c->fine) bufs.push_back(&b);
    for (auto& lvb : c->lev)
      for (auto& b : lvb) bufs.push_back(&b);
    for (DevBuf* b : {&c->slots, &c->active, &c->nactive, &c->freqtab, &c->partials, &c->resid, &c->fstart,
                      &c->rh_idx, &c->rh_val, &c->cinv_a, &c->cinv_b, &c->winv, &c->gm_V, &c->gm_small,
                      &c->gm_part})
      bufs.push_back(b);
    for (DevBuf* b : bufs) {
      saved.push_back({b->p, b->bytes, b->borrowed});
      b->p = nullptr;
      b->bytes = 0;
      b->borrowed = false;
    }
    ws_slots = c->ws_slots;
    ws_levels = c->ws_levels;
    slot_cap = c->slot_cap;
    partial_tiles = c->partial_tiles;
    cinv_key = c->cinv_key;
    cinv_base = c->cinv_base;
    c->ws_slots = c->ws_levels = c->slot_cap = c->partial_tiles = 0;
    c->cinv_key.clear();
    c->cinv_base = nullptr;
  }
  ~WorkspaceStash() {
    (void)hipStreamSynchronize(c->stream);  // nothing may still use the arena's regions
    for (size_t i = 0; i < bufs.size(); ++i) {
      bufs[i]->p = saved[i].p;
      bufs[i]->bytes = saved[i].bytes;
      bufs[i]->borrowed = saved[i].borrowed;
    }
    c->ws_slots = ws_slots;
    c->ws_levels = ws_levels;
    c->slot_cap = slot_cap;
    c->partial_tiles = partial_tiles;
    c->cinv_key = cinv_key;
    c->cinv_base = cinv_base;
  }
};

}  // namespace

int hz_solve_noalloc(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha,
                     int nrhs, const hz_c128* b_dev, hz_c128* u_dev, hz_rhs_info* info) {
  int rc = require_model(c);
  if (rc) return rc;
  HZ_HIP(c, hipSetDevice(c->device));
  void* base = scratch_of(c->device);
  if (c->scratch_status != hipSuccess || !base)
    return fail(c, HZ_ERR_DEVICE, "the scratch array of device %d was not found: %s", c->device,
                hipGetErrorString(c->scratch_status));
  Arena arena;
  arena.base = static_cast<char*>(base);
  arena.cap = HZ_NOALLOC_BYTES;
  {
    WorkspaceStash stash(c);
    c->noalloc = true;
    t_arena = &arena;
    rc = solve_impl(c, o, nfreq, freq_hz, alpha, nrhs, b_dev, u_dev, info);
    t_arena = nullptr;
    c->noalloc = false;
  }
  if (rc == HZ_ERR_NOMEM && arena.wanted > arena.cap)
    return fail(c, HZ_ERR_NOMEM,
                "the solve's workspace exceeds the %zu bytes of the allocation-free call (at least %zu needed)",
                (size_t)HZ_NOALLOC_BYTES, arena.wanted);
  return rc;
}

namespace {
// The misfit, gradient and Gauss-Newton step for sources and receivers given
// as flat node indices (checked by the public calls below).
int misfit_nodes(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nsrc,
                 const std::vector<int>& snodes, const hz_c128* src_amp, int nrec, const std::vector<int>& rnodes,
                 const hz_c128* d_obs_dev, double lambda, double* J, hz_c128* d_cal_dev, hz_rhs_info* info) {
  int rc;
  if (nfreq < 1 || nsrc < 1 || nrec < 1 || !freq_hz || !d_obs_dev || !J)
    return fail(c, HZ_ERR_ARG, "bad misfit arguments");
  if (!(lambda >= 0.0) || !isfinite(lambda)) return fail(c, HZ_ERR_ARG, "lambda must be >= 0");
  HZ_HIP(c, hipSetDevice(c->device));
  const size_t n0 = c->lv[0].n();
  const size_t nb = (size_t)nfreq * nsrc * n0;
  HZ_ALLOC(c, c->misfit_b, nb * sizeof(double2));
  HZ_ALLOC(c, c->misfit_u, nb * sizeof(double2));
  for (int f = 0; f < nfreq; ++f) {
    rc = set_points(c, snodes, src_amp, reinterpret_cast<hz_c128*>(c->misfit_b.as<double2>() + (size_t)f * nsrc * n0));
    if (rc) return rc;
  }
  rc = hz_solve(c, o, nfreq, freq_hz, alpha, nsrc, reinterpret_cast<const hz_c128*>(c->misfit_b.p),
                reinterpret_cast<hz_c128*>(c->misfit_u.p), info);
  if (rc < 0) return rc;
  const int solve_rc = rc;
  const size_t nd = (size_t)nfreq * nsrc * nrec;
  double2* dcal = reinterpret_cast<double2*>(d_cal_dev);
  if (!dcal) {
    HZ_ALLOC(c, c->misfit_d, nd * sizeof(double2));
    dcal = c->misfit_d.as<double2>();
  }
  HZ_ALLOC(c, c->scratch_int, (size_t)nrec * sizeof(int));
  HZ_HIP(c, hipMemcpyAsync(c->scratch_int.p, rnodes.data(), nrec * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, launch_gather(nfreq * nsrc, nrec, c->scratch_int.as<int>(), c->misfit_u.as<double2>(), n0, dcal, c->stream));
  HZ_ALLOC(c, c->misfit_out, 4 * sizeof(double));
  HZ_HIP(c, launch_misfit(nd, reinterpret_cast<const double2*>(d_obs_dev), dcal, n0,
                          c->lv[0].m.as<double>(), lambda, c->misfit_out.as<double>(), c->stream));
  double out[3];
  HZ_HIP(c, hipMemcpyAsync(out, c->misfit_out.p, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  *J = out[0];
  return solve_rc;
}

int gradient_nodes(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nsrc,
                   const std::vector<int>& snodes, const hz_c128* src_amp, int nrec, const std::vector<int>& rnode,
                   const hz_c128* d_obs_dev, double lambda, double* J, double* grad_dev, hz_rhs_info* info) {
  int rc;
  if (nfreq < 1 || nsrc < 1 || nrec < 1 || !freq_hz || !d_obs_dev || !J || !grad_dev)
    return fail(c, HZ_ERR_ARG, "bad gradient arguments");
  if (!(lambda >= 0.0) || !isfinite(lambda)) return fail(c, HZ_ERR_ARG, "lambda must be >= 0");
  for (int f = 0; f < nfreq; ++f)
    if (!(freq_hz[f] > 0.0) || !isfinite(freq_hz[f])) return fail(c, HZ_ERR_ARG, "frequency %d must be positive", f);
  // distinct receiver nodes and, for each, its receivers (in receiver order)
  std::vector<int> order(nrec);
  for (int r = 0; r < nrec; ++r) order[r] = r;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rnode[a] < rnode[b]; });
  std::vector<int> uniq, ptr, idx;
  for (int q = 0; q < nrec; ++q) {
    if (q == 0 || rnode[order[q]] != rnode[order[q - 1]]) {
      uniq.push_back(rnode[order[q]]);
      ptr.push_back(q);
    }
    idx.push_back(order[q]);
  }
  ptr.push_back(nrec);
  const int nuniq = (int)uniq.size();
  HZ_HIP(c, hipSetDevice(c->device));
  const size_t n0 = c->lv[0].n();
  // frequencies per chunk: three wavefield sets (rhs, u, mu) per right-hand side
  int chunk = nfreq;
  if (c->budget) {
    const size_t per_freq = (size_t)nsrc * n0 * sizeof(double2) * (3 + 12);
    chunk = (int)std::max<size_t>(1, std::min<size_t>(nfreq, c->budget / std::max<size_t>(per_freq, 1)));
  }
  const size_t nb = (size_t)chunk * nsrc * n0;
  HZ_ALLOC(c, c->fwi_b, nb * sizeof(double2));
  HZ_ALLOC(c, c->fwi_u, nb * sizeof(double2));
  HZ_ALLOC(c, c->fwi_mu, nb * sizeof(double2));
  HZ_ALLOC(c, c->fwi_d, (size_t)chunk * nsrc * nrec * sizeof(double2));
  HZ_ALLOC(c, c->fwi_int, (size_t)(3 * nrec + 2) * sizeof(int));
  HZ_ALLOC(c, c->fwi_omega, (size_t)nfreq * sizeof(double));
  HZ_ALLOC(c, c->fwi_out, 4 * sizeof(double));
  int* d_uniq = c->fwi_int.as<int>();
  int* d_ptr = d_uniq + nrec;
  int* d_idx = d_ptr + nrec + 1;
  HZ_HIP(c, hipMemcpyAsync(d_uniq, uniq.data(), nuniq * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(d_ptr, ptr.data(), (nuniq + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(d_idx, idx.data(), nrec * sizeof(int), hipMemcpyHostToDevice, c->stream));
  std::vector<double> om(nfreq);
  for (int f = 0; f < nfreq; ++f) om[f] = 2.0 * M_PI * freq_hz[f];
  HZ_HIP(c, hipMemcpyAsync(c->fwi_omega.p, om.data(), nfreq * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  double jdata = 0.0, msum = 0.0;
  int worst = HZ_OK;
  for (int f0 = 0; f0 < nfreq; f0 += chunk) {
    const int nf = std::min(chunk, nfreq - f0);
    for (int f = 0; f < nf; ++f) {
      rc = set_points(c, snodes, src_amp, reinterpret_cast<hz_c128*>(c->fwi_b.as<double2>() + (size_t)f * nsrc * n0));
      if (rc) return rc;
    }
    hz_rhs_info* inf_fwd = info ? info + (size_t)f0 * nsrc : nullptr;
    hz_rhs_info* inf_adj = info ? info + (size_t)(nfreq + f0) * nsrc : nullptr;
    rc = hz_solve(c, o, nf, freq_hz + f0, alpha, nsrc, reinterpret_cast<const hz_c128*>(c->fwi_b.p),
                  reinterpret_cast<hz_c128*>(c->fwi_u.p), inf_fwd);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    const double2* dobs = reinterpret_cast<const double2*>(d_obs_dev) + (size_t)f0 * nsrc * nrec;
    // data misfit of the chunk
    HZ_ALLOC(c, c->scratch_int, (size_t)nrec * sizeof(int));
    HZ_HIP(c, hipMemcpyAsync(c->scratch_int.p, rnode.data(), nrec * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HZ_HIP(c, launch_gather(nf * nsrc, nrec, c->scratch_int.as<int>(), c->fwi_u.as<double2>(), n0,
                            c->fwi_d.as<double2>(), c->stream));
    HZ_HIP(c, launch_misfit((size_t)nf * nsrc * nrec, dobs, c->fwi_d.as<double2>(), n0, c->lv[0].m.as<double>(),
                            0.0, c->fwi_out.as<double>(), c->stream));
    double out[3];
    HZ_HIP(c, hipMemcpyAsync(out, c->fwi_out.p, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    // adjoint sources and solves
    HZ_HIP(c, launch_adjoint_src(nf * nsrc, n0, nuniq, d_uniq, d_ptr, d_idx, nrec, c->fwi_u.as<double2>(), dobs,
                                 c->fwi_b.as<double2>(), c->stream));
    HZ_HIP(c, hipStreamSynchronize(c->stream));
    jdata += out[1];
    msum = out[2];
    rc = hz_solve(c, o, nf, freq_hz + f0, alpha, nsrc, reinterpret_cast<const hz_c128*>(c->fwi_b.p),
                  reinterpret_cast<hz_c128*>(c->fwi_mu.p), inf_adj);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    HZ_HIP(c, launch_grad_accum(c->dim, grid_of(c, 0), nf, nsrc, c->fwi_omega.as<double>() + f0, alpha,
                                c->fwi_u.as<double2>(), c->fwi_mu.as<double2>(), lambda, c->lv[0].m.as<double>(),
                                f0 > 0 ? 1 : 0, grad_dev, c->stream));
  }
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  *J = jdata + lambda * msum;
  return worst;
}

int gn_step_nodes(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nsrc,
                  const std::vector<int>& snodes, const hz_c128* src_amp, int nrec, const std::vector<int>& rnode,
                  const hz_c128* d_obs_dev, double lambda, int cg_iters, double cg_tol, double* J, double* dm_dev,
                  int* cg_done, hz_rhs_info* info) {
  int rc;
  if (nfreq < 1 || nsrc < 1 || nrec < 1 || !freq_hz || !d_obs_dev || !J || !dm_dev || !cg_done || cg_iters < 0)
    return fail(c, HZ_ERR_ARG, "bad Gauss-Newton arguments");
  if (!(lambda >= 0.0) || !isfinite(lambda) || !(cg_tol >= 0.0)) return fail(c, HZ_ERR_ARG, "bad lambda or cg_tol");
  for (int f = 0; f < nfreq; ++f)
    if (!(freq_hz[f] > 0.0) || !isfinite(freq_hz[f])) return fail(c, HZ_ERR_ARG, "frequency %d must be positive", f);
  std::vector<int> order(nrec);
  for (int r = 0; r < nrec; ++r) order[r] = r;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rnode[a] < rnode[b]; });
  std::vector<int> uniq, ptr, idx;
  for (int q = 0; q < nrec; ++q) {
    if (q == 0 || rnode[order[q]] != rnode[order[q - 1]]) {
      uniq.push_back(rnode[order[q]]);
      ptr.push_back(q);
    }
    idx.push_back(order[q]);
  }
  ptr.push_back(nrec);
  const int nuniq = (int)uniq.size();
  HZ_HIP(c, hipSetDevice(c->device));
  const size_t n0 = c->lv[0].n();
  const int nslots = nfreq * nsrc;
  const size_t nb = (size_t)nslots * n0;
  HZ_ALLOC(c, c->fwi_b, nb * sizeof(double2));
  HZ_ALLOC(c, c->fwi_u, nb * sizeof(double2));
  HZ_ALLOC(c, c->fwi_mu, nb * sizeof(double2));
  HZ_ALLOC(c, c->fwi_d, (size_t)nslots * nrec * sizeof(double2));
  HZ_ALLOC(c, c->fwi_int, (size_t)(3 * nrec + 2) * sizeof(int));
  HZ_ALLOC(c, c->fwi_omega, (size_t)nfreq * sizeof(double));
  HZ_ALLOC(c, c->fwi_out, 4 * sizeof(double));
  HZ_ALLOC(c, c->gn_g, n0 * sizeof(double));
  HZ_ALLOC(c, c->gn_r, n0 * sizeof(double));
  HZ_ALLOC(c, c->gn_p, n0 * sizeof(double));
  HZ_ALLOC(c, c->gn_hp, n0 * sizeof(double));
  HZ_ALLOC(c, c->gn_state, 4 * sizeof(double));
  int* d_uniq = c->fwi_int.as<int>();
  int* d_ptr = d_uniq + nrec;
  int* d_idx = d_ptr + nrec + 1;
  HZ_HIP(c, hipMemcpyAsync(d_uniq, uniq.data(), nuniq * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(d_ptr, ptr.data(), (nuniq + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(d_idx, idx.data(), nrec * sizeof(int), hipMemcpyHostToDevice, c->stream));
  std::vector<double> om(nfreq);
  for (int f = 0; f < nfreq; ++f) om[f] = 2.0 * M_PI * freq_hz[f];
  HZ_HIP(c, hipMemcpyAsync(c->fwi_omega.p, om.data(), nfreq * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  double2* B = c->fwi_b.as<double2>();
  double2* U = c->fwi_u.as<double2>();
  double2* MU = c->fwi_mu.as<double2>();
  double2* D = c->fwi_d.as<double2>();
  const double* omg = c->fwi_omega.as<double>();
  const Grid g0 = grid_of(c, 0);
  int worst = HZ_OK;
  // forward fields, kept for every Born product
  for (int f = 0; f < nfreq; ++f) {
    rc = set_points(c, snodes, src_amp, reinterpret_cast<hz_c128*>(B + (size_t)f * nsrc * n0));
    if (rc) return rc;
  }
  rc = hz_solve(c, o, nfreq, freq_hz, alpha, nsrc, reinterpret_cast<const hz_c128*>(B), reinterpret_cast<hz_c128*>(U),
                info);
  if (rc < 0) return rc;
  worst = std::max(worst, rc);
  HZ_ALLOC(c, c->scratch_int, (size_t)nrec * sizeof(int));
  HZ_HIP(c, hipMemcpyAsync(c->scratch_int.p, rnode.data(), nrec * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, launch_gather(nslots, nrec, c->scratch_int.as<int>(), U, n0, D, c->stream));
  HZ_HIP(c, launch_misfit((size_t)nslots * nrec, reinterpret_cast<const double2*>(d_obs_dev), D, n0,
                          c->lv[0].m.as<double>(), lambda, c->fwi_out.as<double>(), c->stream));
  double out[3];
  HZ_HIP(c, hipMemcpyAsync(out, c->fwi_out.p, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  // gradient g = -2 Re sum delta u mu + 2 lambda m
  HZ_HIP(c, launch_adjoint_src(nslots, n0, nuniq, d_uniq, d_ptr, d_idx, nrec, U,
                               reinterpret_cast<const double2*>(d_obs_dev), B, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  *J = out[0];
  rc = hz_solve(c, o, nfreq, freq_hz, alpha, nsrc, reinterpret_cast<const hz_c128*>(B), reinterpret_cast<hz_c128*>(MU),
                nullptr);
  if (rc < 0) return rc;
  worst = std::max(worst, rc);
  double* gv = c->gn_g.as<double>();
  double* xr = c->gn_r.as<double>();
  double* xp = c->gn_p.as<double>();
  double* hp = c->gn_hp.as<double>();
  double* stt = c->gn_state.as<double>();
  HZ_HIP(c, launch_grad_accum(c->dim, g0, nfreq, nsrc, omg, alpha, U, MU, lambda, c->lv[0].m.as<double>(), 0, gv,
                              c->stream));
  // conjugate gradients on H dm = -g; each product is one Born and one adjoint batch
  HZ_HIP(c, launch_cg(0, n0, gv, nullptr, dm_dev, xr, xp, stt, cg_tol, c->stream));
  int it = 0;
  while (it < cg_iters) {
    double st3[3];
    HZ_HIP(c, hipMemcpyAsync(st3, stt, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HZ_HIP(c, hipStreamSynchronize(c->stream));
    if (st3[2] != 0.0) break;
    HZ_HIP(c, launch_born_src(c->dim, g0, nslots, nsrc, omg, alpha, U, xp, B, c->stream));
    rc = hz_solve(c, o, nfreq, freq_hz, alpha, nsrc, reinterpret_cast<const hz_c128*>(B),
                  reinterpret_cast<hz_c128*>(MU), nullptr);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    HZ_HIP(c, launch_gather(nslots, nrec, c->scratch_int.as<int>(), MU, n0, D, c->stream));
    HZ_HIP(c, launch_adjoint_data(nslots, n0, nuniq, d_uniq, d_ptr, d_idx, nrec, D, B, c->stream));
    rc = hz_solve(c, o, nfreq, freq_hz, alpha, nsrc, reinterpret_cast<const hz_c128*>(B),
                  reinterpret_cast<hz_c128*>(MU), nullptr);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    HZ_HIP(c, launch_grad_accum(c->dim, g0, nfreq, nsrc, omg, alpha, U, MU, lambda, xp, 0, hp, c->stream));
    HZ_HIP(c, launch_cg(1, n0, gv, hp, dm_dev, xr, xp, stt, cg_tol, c->stream));
    ++it;
  }
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  *cg_done = it;
  return worst;
}

// flat node indices of n points given per axis (iy null for a 1D or 2D
// grid); what names the points in the error message
int node_list(hz_ctx* c, int n, const int* iz, const int* iy, const int* ix, const char* what,
              std::vector<int>& nodes) {
  if (n < 1 || !iz || !ix || (c->dim == 3 && !iy)) return fail(c, HZ_ERR_ARG, "bad %s arguments", what);
  nodes.resize(n);
  for (int k = 0; k < n; ++k) {
    const int y = c->dim == 3 ? iy[k] : 0;
    if (iz[k] < 0 || iz[k] >= c->nz || y < 0 || y >= c->ny || ix[k] < 0 || ix[k] >= c->nx)
      return fail(c, HZ_ERR_ARG, "%s %d is outside the grid", what, k);
    nodes[k] = (iz[k] * c->ny + y) * c->nx + ix[k];
  }
  return HZ_OK;
}

// the model, its dimension and the source and receiver lists of a public call
int fwi_points(hz_ctx* c, bool three_d, int nsrc, const int* src_iz, const int* src_iy, const int* src_ix,
               int nrec, const int* rec_iz, const int* rec_iy, const int* rec_ix, std::vector<int>& snodes,
               std::vector<int>& rnodes) {
  int rc = require_model(c);
  if (rc) return rc;
  if (three_d && c->dim != 3) return fail(c, HZ_ERR_ARG, "the model is not 3D: use the call without _3d");
  if (!three_d && c->dim == 3) return fail(c, HZ_ERR_ARG, "the model is 3D: use the _3d call");
  rc = node_list(c, nsrc, src_iz, src_iy, src_ix, "source", snodes);
  if (rc) return rc;
  return node_list(c, nrec, rec_iz, rec_iy, rec_ix, "receiver", rnodes);
}
}  // namespace

int hz_misfit(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha,
              int nsrc, const int* src_iz, const int* src_ix, const hz_c128* src_amp, int nrec,
              const int* rec_iz, const int* rec_ix, const hz_c128* d_obs_dev, double lambda,
              double* J, hz_c128* d_cal_dev, hz_rhs_info* info) {
  std::vector<int> sn, rn;
  int rc = fwi_points(c, false, nsrc, src_iz, nullptr, src_ix, nrec, rec_iz, nullptr, rec_ix, sn, rn);
  if (rc) return rc;
  return misfit_nodes(c, o, nfreq, freq_hz, alpha, nsrc, sn, src_amp, nrec, rn, d_obs_dev, lambda, J, d_cal_dev,
                      info);
}

int hz_misfit_3d(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nsrc,
                 const int* src_iz, const int* src_iy, const int* src_ix, const hz_c128* src_amp, int nrec,
                 const int* rec_iz, const int* rec_iy, const int* rec_ix, const hz_c128* d_obs_dev, double lambda,
                 double* J, hz_c128* d_cal_dev, hz_rhs_info* info) {
  std::vector<int> sn, rn;
  int rc = fwi_points(c, true, nsrc, src_iz, src_iy, src_ix, nrec, rec_iz, rec_iy, rec_ix, sn, rn);
  if (rc) return rc;
  return misfit_nodes(c, o, nfreq, freq_hz, alpha, nsrc, sn, src_amp, nrec, rn, d_obs_dev, lambda, J, d_cal_dev,
                      info);
}

int hz_gradient(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha,
                int nsrc, const int* src_iz, const int* src_ix, const hz_c128* src_amp, int nrec,
                const int* rec_iz, const int* rec_ix, const hz_c128* d_obs_dev, double lambda, double* J,
                double* grad_dev, hz_rhs_info* info) {
  std::vector<int> sn, rn;
  int rc = fwi_points(c, false, nsrc, src_iz, nullptr, src_ix, nrec, rec_iz, nullptr, rec_ix, sn, rn);
  if (rc) return rc;
  return gradient_nodes(c, o, nfreq, freq_hz, alpha, nsrc, sn, src_amp, nrec, rn, d_obs_dev, lambda, J, grad_dev,
                        info);
}

int hz_gradient_3d(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nsrc,
                   const int* src_iz, const int* src_iy, const int* src_ix, const hz_c128* src_amp, int nrec,
                   const int* rec_iz, const int* rec_iy, const int* rec_ix, const hz_c128* d_obs_dev,
                   double lambda, double* J, double* grad_dev, hz_rhs_info* info) {
  std::vector<int> sn, rn;
  int rc = fwi_points(c, true, nsrc, src_iz, src_iy, src_ix, nrec, rec_iz, rec_iy, rec_ix, sn, rn);
  if (rc) return rc;
  return gradient_nodes(c, o, nfreq, freq_hz, alpha, nsrc, sn, src_amp, nrec, rn, d_obs_dev, lambda, J, grad_dev,
                        info);
}

int hz_gn_step(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha,
               int nsrc, const int* src_iz, const int* src_ix, const hz_c128* src_amp, int nrec,
               const int* rec_iz, const int* rec_ix, const hz_c128* d_obs_dev, double lambda, int cg_iters,
               double cg_tol, double* J, double* dm_dev, int* cg_done, hz_rhs_info* info) {
  std::vector<int> sn, rn;
  int rc = fwi_points(c, false, nsrc, src_iz, nullptr, src_ix, nrec, rec_iz, nullptr, rec_ix, sn, rn);
  if (rc) return rc;
  return gn_step_nodes(c, o, nfreq, freq_hz, alpha, nsrc, sn, src_amp, nrec, rn, d_obs_dev, lambda, cg_iters,
                       cg_tol, J, dm_dev, cg_done, info);
}

int hz_gn_step_3d(hz_ctx* c, const hz_solve_opts* o, int nfreq, const double* freq_hz, double alpha, int nsrc,
                  const int* src_iz, const int* src_iy, const int* src_ix, const hz_c128* src_amp, int nrec,
                  const int* rec_iz, const int* rec_iy, const int* rec_ix, const hz_c128* d_obs_dev,
                  double lambda, int cg_iters, double cg_tol, double* J, double* dm_dev, int* cg_done,
                  hz_rhs_info* info) {
  std::vector<int> sn, rn;
  int rc = fwi_points(c, true, nsrc, src_iz, src_iy, src_ix, nrec, rec_iz, rec_iy, rec_ix, sn, rn);
  if (rc) return rc;
  return gn_step_nodes(c, o, nfreq, freq_hz, alpha, nsrc, sn, src_amp, nrec, rn, d_obs_dev, lambda, cg_iters,
                       cg_tol, J, dm_dev, cg_done, info);
}

int hz_apply(hz_ctx* c, int op, int level, double freq_hz, double alpha, double beta1, double beta2,
             int nrhs, const hz_c128* x_dev, hz_c128* y_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  if (op != 0 && op != 1) return fail(c, HZ_ERR_ARG, "op must be 0 (B) or 1 (M)");
  if (level < 0 || level >= c->maxlev) return fail(c, HZ_ERR_SHAPE, "level %d does not exist", level);
  if (!x_dev || !y_dev) return fail(c, HZ_ERR_ARG, "null vector");
  HZ_HIP(c, hipSetDevice(c->device));
  if ((rc = setup_debug_batch(c, nrhs, freq_hz, alpha, beta1, beta2, nullptr, 0)) != HZ_OK) return rc;
  HZ_HIP(c, launch_apply(c->dim, grid_of(c, level), level, op, batch_of(c), nrhs,
                         reinterpret_cast<const double2*>(x_dev), reinterpret_cast<double2*>(y_dev),
                         c->lv[level].n(), c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

int hz_smooth(hz_ctx* c, int level, double freq_hz, double beta1, double beta2, double w, int nrhs,
              const hz_c128* b_dev, const hz_c128* u_in_dev, hz_c128* u_out_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  if (level < 0 || level >= c->maxlev) return fail(c, HZ_ERR_SHAPE, "level %d does not exist", level);
  if (!b_dev || !u_out_dev || u_in_dev == u_out_dev) return fail(c, HZ_ERR_ARG, "bad vectors");
  if (!(w > 0.0)) return fail(c, HZ_ERR_ARG, "w must be positive");
  HZ_HIP(c, hipSetDevice(c->device));
  if ((rc = setup_debug_batch(c, nrhs, freq_hz, 0.0, beta1, beta2, nullptr, 0)) != HZ_OK) return rc;
  HZ_HIP(c, launch_smooth(c->dim, grid_of(c, level), level, w, batch_of(c), nrhs,
                          reinterpret_cast<const double2*>(b_dev), reinterpret_cast<const double2*>(u_in_dev),
                          reinterpret_cast<double2*>(u_out_dev), c->lv[level].n(), c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

int hz_restrict(hz_ctx* c, int level, double freq_hz, double beta1, double beta2, int nrhs,
                const hz_c128* b_dev, const hz_c128* u_dev, hz_c128* bc_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  if (level < 0 || level + 1 >= c->maxlev) return fail(c, HZ_ERR_SHAPE, "level %d has no coarser level", level);
  if (!b_dev || !u_dev || !bc_dev) return fail(c, HZ_ERR_ARG, "null vector");
  HZ_HIP(c, hipSetDevice(c->device));
  if ((rc = setup_debug_batch(c, nrhs, freq_hz, 0.0, beta1, beta2, nullptr, 0)) != HZ_OK) return rc;
  HZ_HIP(c, launch_restrict(c->dim, grid_of(c, level), grid_of(c, level + 1), batch_of(c), nrhs,
                            reinterpret_cast<const double2*>(b_dev), reinterpret_cast<const double2*>(u_dev),
                            reinterpret_cast<double2*>(bc_dev), c->lv[level].n(), c->lv[level + 1].n(),
                            c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

int hz_prolong(hz_ctx* c, int level, int nrhs, const hz_c128* e_dev, hz_c128* u_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  if (level < 0 || level + 1 >= c->maxlev) return fail(c, HZ_ERR_SHAPE, "level %d has no coarser level", level);
  if (!e_dev || !u_dev) return fail(c, HZ_ERR_ARG, "null vector");
  HZ_HIP(c, hipSetDevice(c->device));
  if ((rc = setup_debug_batch(c, nrhs, 1.0, 0.0, 1.0, 0.5, nullptr, 0)) != HZ_OK) return rc;
  double2* u = reinterpret_cast<double2*>(u_dev);
  HZ_HIP(c, launch_prolong(c->dim, grid_of(c, level), grid_of(c, level + 1), batch_of(c), nrhs,
                           reinterpret_cast<const double2*>(e_dev), u, u, c->lv[level].n(),
                           c->lv[level + 1].n(), c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

int hz_precond(hz_ctx* c, const hz_solve_opts* o, double freq_hz, int nrhs, const hz_c128* b_dev,
               hz_c128* u_dev) {
  int rc = require_model(c);
  if (rc) return rc;
  hz_solve_opts d;
  if (!o) {
    hz_default_opts(&d);
    o = &d;
  }
  if (!b_dev || !u_dev || nrhs < 1) return fail(c, HZ_ERR_ARG, "bad vectors");
  if (!(freq_hz > 0.0) || !isfinite(freq_hz)) return fail(c, HZ_ERR_ARG, "frequency must be positive");
  if ((rc = check_opts(c, o)) != HZ_OK) return rc;
  HZ_HIP(c, hipSetDevice(c->device));
  int levels = 1;
  std::vector<std::vector<double>> wj(1, std::vector<double>(kMaxLevels, 0.0));
  if (o->precond == HZ_PRECOND_MG) {
    if ((rc = make_plan(c, o, 2.0 * M_PI * freq_hz, &levels, wj[0].data())) != HZ_OK)
      return fail(c, rc, "cannot plan the V-cycle: more levels than the grid allows, or an exactly solved "
                         "coarsest level above %d unknowns", kCoarseMax);
  }
  if ((rc = ensure_workspace(c, nrhs, levels)) != HZ_OK) return rc;
  if ((rc = setup_freqs(c, o, 1, &freq_hz, 0.0, levels, wj)) != HZ_OK) return rc;
  if ((rc = reset_slots(c, nrhs, nrhs)) != HZ_OK) return rc;
  const Cycle cy{levels, o->nu1, o->nu2, o->precond, o->autotune, o->chunk_rows,
                 c->any_coarse_jacobi ? o->coarse_sweeps : 0, o->plain, o->plain || (c->has_rho && c->dim != 2)};
  HZ_HIP(c, precond_apply(c, cy, nrhs, reinterpret_cast<const double2*>(b_dev), reinterpret_cast<double2*>(u_dev)));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  return HZ_OK;
}

int hz_timing_start(hz_ctx* c, unsigned mask) {
  if (!c) return HZ_ERR_ARG;
  if (mask >> HZ_KERNEL_CLASSES) return fail(c, HZ_ERR_ARG, "unknown kernel class in mask 0x%x", mask);
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  fold_timing(c);
  c->timing_mask = mask;
  for (int k = 0; k < HZ_KERNEL_CLASSES; ++k) {
    c->t_launches[k] = 0;
    c->t_ms[k] = 0.0;
  }
  return HZ_OK;
}

int hz_timing_read(hz_ctx* c, int kernel, int* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return HZ_ERR_ARG;
  if (kernel < 0 || kernel >= HZ_KERNEL_CLASSES) return fail(c, HZ_ERR_ARG, "unknown kernel class %d", kernel);
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  fold_timing(c);
  *launches = (int)c->t_launches[kernel];
  *total_ms = c->t_ms[kernel];
  return HZ_OK;
}

const char* hz_status_str(int status) {
  switch (status) {
    case HZ_OK: return "ok";
    case HZ_WARN_NOCONV: return "some right-hand side did not converge";
    case HZ_ERR_ARG: return "invalid argument";
    case HZ_ERR_SHAPE: return "grid cannot be coarsened as requested";
    case HZ_ERR_NOMEM: return "out of device memory or workspace budget";
    case HZ_ERR_DEVICE: return "HIP runtime error";
    case HZ_ERR_STATE: return "no model set";
    default: return "unknown status";
  }
}

const char* hz_last_error(const hz_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ---------------------------------------------------------------- continuous-batching engine
struct hz_engine {
  hz_ctx* c = nullptr;
  int lanes = 0, width = 0, L = 0;
  hz_solve_opts o{};
  Cycle cy{};
  DevBuf B, X;      // right-hand sides and iterates of every slot, [lanes * width][n]
  DevBuf cwork;     // Gauss-Jordan work matrix of one lane
  DevBuf list, count;  // a short active list (slots being started or finished)
  DevBuf chk;       // model check output
  int* fst_host = nullptr;  // pinned, [kRing][lanes + 1]: per-lane ranges of each summary's list
  std::vector<FreqTab> ft;  // host copy of the lane table
  size_t winv_per_lane = 0, nc = 0;
  struct Part {
    int lane, fi, off, cnt;  // right-hand sides off .. off + cnt - 1 of frequency fi
  };
  struct Running {
    hz::EngineJob job;
    std::vector<Part> parts;
  };
  std::vector<Running> running;
  std::vector<int> free_lanes;
  std::string err;
};

namespace {

size_t level_nodes(int nz, int nx, int l) {
  for (int k = 0; k < l; ++k) {
    nz = coarse_n(nz);
    nx = coarse_n(nx);
  }
  return (size_t)nz * nx;
}

int engine_levels(int nz, int nx, const hz_solve_opts* o) {
  const int L = grid_default_levels(2, nz, nx);
  return o->levels > 0 ? std::min(o->levels, grid_max_levels(2, nz, nx)) : L;
}

// Copies a request's model into a lane's model rows (every level), and its
// smallest and largest slowness.
int engine_model(hz_engine* e, int lane, const double* m_dev, double* mmin, double* mmax) {
  hz_ctx* c = e->c;
  const size_t n0 = c->lv[0].n();
  double* m0 = c->lv[0].m.as<double>() + (size_t)lane * c->lv[0].mstride;
  HZ_HIP(c, hipMemcpyAsync(m0, m_dev, n0 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  for (int l = 1; l < e->L; ++l) {
    Grid gf = grid_of(c, l - 1);
    gf.m += (size_t)lane * gf.mstride;
    gf.mstride = 0;
    HZ_HIP(c, launch_inject(gf, 2, c->lv[l].m.as<double>() + (size_t)lane * c->lv[l].mstride, c->stream));
  }
  HZ_HIP(c, launch_check_model(n0, m0, e->chk.as<double>(), c->stream));
  double out3[3];
  HZ_HIP(c, hipMemcpyAsync(out3, e->chk.p, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  if (out3[2] > 0.0) return fail(c, HZ_ERR_ARG, "slowness has %.0f entries that are not finite and positive", out3[2]);
  *mmin = out3[0];
  *mmax = out3[1];
  return HZ_OK;
}

// The lane table entry of one (request, frequency): plan weights, w / D
// tables, coarse inverse or coarse smoothing, the model it reads.
int engine_lane_setup(hz_engine* e, int lane, int model, double mmin, double mmax, double freq_hz, double alpha) {
  hz_ctx* c = e->c;
  FreqTab& f = e->ft[lane];
  memset(&f, 0, sizeof f);
  f.omega = 2.0 * M_PI * freq_hz;
  f.sB_re = 1.0;
  f.sB_im = -alpha;
  f.sM_re = e->o.beta1;
  f.sM_im = -e->o.beta2;
  f.model = model;
  int L = 0;
  double w[kMaxLevels] = {};
  hz_solve_opts po = e->o;
  po.levels = e->L;
  int rc = plan_grid(2, c->nz, 1, c->nx, c->maxlev, e->L, c->h, mmin, mmax, &po, f.omega, &L, w);
  if (rc != HZ_OK || L != e->L) return fail(c, HZ_ERR_SHAPE, "cannot plan the V-cycle of a lane");
  for (int l = 0; l < L - 1; ++l) f.wj[l] = w[l];
  double2* wp = c->winv.as<double2>() + (size_t)lane * e->winv_per_lane;
  for (int l = 0; l < L - 1; ++l) {
    Grid g = grid_of(c, l);
    g.m += (size_t)model * g.mstride;
    g.mstride = 0;
    HZ_HIP(c, launch_winv(2, g, f.omega, f.sM_re, f.sM_im, f.wj[l], wp, c->stream));
    f.winv[l] = wp;
    wp += c->lv[l].n();
  }
  const int cl = L - 1;
  f.coarse_jacobi = !coarse_is_exact(&e->o, L, c->lv[cl].h, mmin, f.omega) ? 1 : 0;
  double2* cinv = c->cinv_a.as<double2>() + (size_t)lane * e->nc * e->nc;
  f.cinv = cinv;
  HZ_HIP(c, hipMemcpyAsync(c->freqtab.as<FreqTab>() + lane, &f, sizeof f, hipMemcpyHostToDevice, c->stream));
  if (!f.coarse_jacobi) {
    Grid g = grid_of(c, cl);
    g.m += (size_t)model * g.mstride;
    g.mstride = 0;
    double2* work = e->cwork.as<double2>();
    HZ_HIP(c, launch_assemble_dense(2, g, 1, c->freqtab.as<FreqTab>() + lane, work, c->stream));
    double2* src = work;
    double2* dst = cinv;
    for (size_t k = 0; k < e->nc; ++k) {
      HZ_HIP(c, launch_gj_step((int)e->nc, 1, (int)k, src, dst, c->stream));
      std::swap(src, dst);
    }
    if (src != cinv)
      HZ_HIP(c, hipMemcpyAsync(cinv, src, e->nc * e->nc * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
  }
  return HZ_OK;
}

// The slots k0 .. k0 + cnt - 1 as a short active list (a batch over them).
int engine_list(hz_engine* e, const std::vector<int>& slots, Batch* lb) {
  hz_ctx* c = e->c;
  const int n = (int)slots.size();
  HZ_HIP(c, hipMemcpyAsync(e->list.p, slots.data(), n * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipMemcpyAsync(e->count.p, &n, sizeof(int), hipMemcpyHostToDevice, c->stream));
  *lb = batch_of(c);
  lb->active = e->list.as<int>();
  lb->nactive = e->count.as<int>();
  return HZ_OK;
}

}  // namespace

namespace hz {

size_t engine_bytes(int nz, int nx, int lanes, int width, const hz_solve_opts* o) {
  const int L = engine_levels(nz, nx, o);
  const size_t slots = (size_t)lanes * width;
  const size_t z = sizeof(double2);
  size_t bytes = 0;
  const size_t n0 = (size_t)nz * nx;
  for (int l = 0; l < L; ++l) bytes += lanes * level_nodes(nz, nx, l) * sizeof(double);  // models
  bytes += (size_t)kNumFine * slots * fine_nodes(2, nz, 1, nx) * z;  // Krylov vectors
  bytes += (size_t)2 * slots * n0 * z;                               // right-hand sides, iterates
  for (int l = 1; l < L; ++l) bytes += (size_t)kNumLevelVec * slots * level_nodes(nz, nx, l) * z;
  for (int l = 0; l + 1 < L; ++l) bytes += lanes * level_nodes(nz, nx, l) * z;  // w / D tables
  const size_t nc = level_nodes(nz, nx, L - 1);
  bytes += (lanes + 1) * nc * nc * z;  // coarse inverses and the work matrix
  const Tiles t = grid_tiles(nz, nx, 2);
  const int tiles = std::max({t.per_slot, reduce_tiles(nz, nx, 2), vec_tiles(n0)});
  bytes += slots * ((size_t)tiles * kPartialWidth * sizeof(double) + sizeof(Slot) + kShadowMax * (sizeof(int) + z) +
                    2 * sizeof(double) + 2 * sizeof(int));
  bytes += lanes * sizeof(FreqTab) + (lanes + 1) * sizeof(int) + 4096;
  return bytes;
}

int engine_create(hz_engine** out, int device, void* stream, int nz, int nx, double h, int lanes, int width,
                  const hz_solve_opts* o) {
  if (!out || !o || nz < 5 || nx < 5 || !(h > 0.0) || lanes < 1 || width < 1) return HZ_ERR_ARG;
  *out = nullptr;
  if (o->krylov != HZ_BICGSTAB || o->precond != HZ_PRECOND_MG || o->plain) return HZ_ERR_ARG;
  hz_engine* e = new hz_engine();
  const hz_ctx_opts co{device, stream, 0};
  int rc = hz_create(&e->c, &co);
  if (rc != HZ_OK) {
    delete e;
    return rc;
  }
  hz_ctx* c = e->c;
  e->lanes = lanes;
  e->width = width;
  e->o = *o;
  e->o.jacobi_w_level = nullptr;
  e->L = engine_levels(nz, nx, o);
  auto bail = [&](int code) {
    e->err = c->err;
    engine_destroy(e);
    return code;
  };
  // the grid of every level, one model row per lane
  c->dim = 2;
  c->nz = nz;
  c->ny = 1;
  c->nx = nx;
  c->h = h;
  c->maxlev = grid_max_levels(2, nz, nx);
  if ((rc = check_opts(c, &e->o)) != HZ_OK) return bail(rc);
  if (e->L < 2) return bail(fail(c, HZ_ERR_SHAPE, "the engine needs at least two levels"));
  for (int l = 0; l < e->L; ++l) {
    LevelInfo& lv = c->lv[l];
    lv.nz = l == 0 ? nz : coarse_n(c->lv[l - 1].nz);
    lv.nx = l == 0 ? nx : coarse_n(c->lv[l - 1].nx);
    lv.ny = 1;
    lv.h = l == 0 ? h : 2.0 * c->lv[l - 1].h;
    lv.mstride = lv.n();
    if (lv.m.ensure((size_t)lanes * lv.n() * sizeof(double)) != hipSuccess) return bail(HZ_ERR_NOMEM);
  }
  e->nc = c->lv[e->L - 1].n();
  if (coarse_is_exact(&e->o, e->L, c->lv[e->L - 1].h, 0.0, 1.0) && e->nc > (size_t)kCoarseMax)
    return bail(fail(c, HZ_ERR_SHAPE, "coarsest level above %d unknowns", kCoarseMax));
  const int nslots = lanes * width;
  if ((rc = ensure_workspace(c, nslots, e->L)) != HZ_OK) return bail(rc);
  const size_t n0 = c->lv[0].n();
  for (int l = 0; l + 1 < e->L; ++l) e->winv_per_lane += c->lv[l].n();
  if (c->winv.ensure((size_t)lanes * e->winv_per_lane * sizeof(double2)) != hipSuccess ||
      c->cinv_a.ensure((size_t)lanes * e->nc * e->nc * sizeof(double2)) != hipSuccess ||
      e->cwork.ensure(e->nc * e->nc * sizeof(double2)) != hipSuccess ||
      c->freqtab.ensure((size_t)lanes * sizeof(FreqTab)) != hipSuccess ||
      c->fstart.ensure((size_t)(lanes + 1) * sizeof(int)) != hipSuccess ||
      e->B.ensure((size_t)nslots * n0 * sizeof(double2)) != hipSuccess ||
      e->X.ensure((size_t)nslots * n0 * sizeof(double2)) != hipSuccess ||
      e->list.ensure((size_t)nslots * sizeof(int)) != hipSuccess || e->count.ensure(sizeof(int)) != hipSuccess ||
      e->chk.ensure(4 * sizeof(double)) != hipSuccess)
    return bail(fail(c, HZ_ERR_NOMEM, "engine buffers"));
  void* fh = nullptr;
  if (hipHostMalloc(&fh, (size_t)kRing * (lanes + 1) * sizeof(int)) != hipSuccess) return bail(HZ_ERR_NOMEM);
  e->fst_host = static_cast<int*>(fh);
  e->ft.assign(lanes, FreqTab{});
  for (int k = 0; k < lanes; ++k) {
    e->ft[k].model = k;
    e->free_lanes.push_back(lanes - 1 - k);  // handed out from the back: lane 0 first
  }
  HZ_HIP(c, hipMemcpyAsync(c->freqtab.p, e->ft.data(), lanes * sizeof(FreqTab), hipMemcpyHostToDevice, c->stream));
  // every slot idle (not in any list) until a lane is given to a request
  std::vector<Slot> sl(nslots);
  for (int i = 0; i < nslots; ++i) {
    memset(&sl[i], 0, sizeof(Slot));
    sl[i].status = kConverged;
    sl[i].freq = i / width;
    sl[i].rh_nnz = -1;
  }
  HZ_HIP(c, hipMemcpyAsync(c->slots.p, sl.data(), nslots * sizeof(Slot), hipMemcpyHostToDevice, c->stream));
  const int zero = 0;
  HZ_HIP(c, hipMemcpyAsync(c->nactive.p, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
  HZ_HIP(c, hipStreamSynchronize(c->stream));
  c->cur_nfreq = lanes;
  c->cur_nrhs = width;
  e->cy = Cycle{e->L, e->o.nu1, e->o.nu2, HZ_PRECOND_MG, e->o.autotune, e->o.chunk_rows, e->o.coarse_sweeps, 0};
  *out = e;
  return HZ_OK;
}

void engine_destroy(hz_engine* e) {
  if (!e) return;
  if (e->c) {
    (void)hipSetDevice(e->c->device);
    (void)hipStreamSynchronize(e->c->stream);
  }
  if (e->fst_host) (void)hipHostFree(e->fst_host);
  e->B.release();
  e->X.release();
  e->cwork.release();
  e->list.release();
  e->count.release();
  e->chk.release();
  hz_destroy(e->c);
  delete e;
}

size_t engine_allocated(const hz_engine* e) {
  const hz_ctx* c = e->c;
  size_t b = e->B.bytes + e->X.bytes + e->cwork.bytes + e->list.bytes + e->count.bytes + e->chk.bytes;
  for (const auto& v : c->fine) b += v.bytes;
  for (const auto& lv : c->lev)
    for (const auto& v : lv) b += v.bytes;
  for (const auto& lv : c->lv) b += lv.m.bytes;
  for (const DevBuf* v : {&c->slots, &c->active, &c->nactive, &c->freqtab, &c->partials, &c->resid, &c->fstart,
                          &c->rh_idx, &c->rh_val, &c->cinv_a, &c->cinv_b, &c->winv})
    b += v->bytes;
  return b;
}

const char* engine_error(const hz_engine* e) { return e ? (e->err.empty() ? e->c->err.c_str() : e->err.c_str()) : ""; }

int engine_run(hz_engine* e, EngineHooks& hooks) {
  hz_ctx* c = e->c;
  HZ_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const int nslots = e->lanes * e->width;
  const int W = e->width;
  const size_t n0 = c->lv[0].n();
  BicgIter it(c, &e->o, e->cy, e->X.as<double2>());
  const Batch bt = it.bt;
  double2* Bv = e->B.as<double2>();
  double2* Xv = e->X.as<double2>();

  long long seq = 0, restart_seq = -1, admit_seq = -1;
  std::deque<std::pair<long long, int>> pending;
  int ring_next = 0;
  auto close_unit = [&]() -> int {
    const int k = ring_next;
    ring_next = (ring_next + 1) % kRing;
    HZ_HIP(c, launch_compact(nslots, W, e->lanes, bt.slots, c->active.as<int>(), c->nactive.as<int>(),
                             c->fstart.as<int>(), c->ring_dev + k, 0, st));
    HZ_HIP(c, hipMemcpyAsync(e->fst_host + (size_t)k * (e->lanes + 1), c->fstart.p, (e->lanes + 1) * sizeof(int),
                             hipMemcpyDeviceToHost, st));
    HZ_HIP(c, hipEventRecord(c->ev[k], st));
    pending.emplace_back(seq++, k);
    return HZ_OK;
  };
  // A finished job: pending iterate terms, true residuals, the result.
  auto finish = [&](hz_engine::Running& run) -> int {
    const EngineJob& jb = run.job;
    std::vector<int> sl;
    std::vector<int> at;  // info index of each listed slot
    for (const auto& pt : run.parts) {
      HZ_HIP(c, launch_bicg_flush(n0, pt.cnt, bt, 0, Xv, it.phr[0], it.shr[0], n0, st, pt.lane * W));
      HZ_HIP(c, hipMemcpyAsync(jb.u_dev + ((size_t)pt.fi * jb.nrhs + pt.off) * n0, Xv + (size_t)pt.lane * W * n0,
                               (size_t)pt.cnt * n0 * sizeof(double2), hipMemcpyDeviceToDevice, st));
      for (int k = 0; k < pt.cnt; ++k) {
        sl.push_back(pt.lane * W + k);
        at.push_back(pt.fi * jb.nrhs + pt.off + k);
      }
    }
    Batch lb;
    int rc = engine_list(e, sl, &lb);
    if (rc) return rc;
    HZ_HIP(c, launch_true_residual(2, grid_of(c, 0), lb, (int)sl.size(), it.rd, Bv, Xv, c->resid.as<double>(), n0, st));
    std::vector<Slot> rec(nslots);
    std::vector<double> res(2 * (size_t)nslots);
    HZ_HIP(c, hipMemcpyAsync(rec.data(), c->slots.p, nslots * sizeof(Slot), hipMemcpyDeviceToHost, st));
    HZ_HIP(c, hipMemcpyAsync(res.data(), c->resid.p, 2 * nslots * sizeof(double), hipMemcpyDeviceToHost, st));
    HZ_HIP(c, hipStreamSynchronize(st));
    std::vector<hz_rhs_info> info(sl.size());
    int any_fail = 0;
    for (size_t i = 0; i < sl.size(); ++i) {
      const Slot& sr = rec[sl[i]];
      int stt = sr.status;
      if (stt == kActive) stt = kMaxit;
      if (stt == kRestart) stt = kBreakdown;
      if (stt != kConverged) any_fail = 1;
      hz_rhs_info& in = info[at[i]];
      in.status = stt;
      in.iters = sr.iters;
      const double r2 = res[2 * (size_t)sl[i]], b2 = res[2 * (size_t)sl[i] + 1];
      in.relres = b2 > 0.0 ? sqrt(r2) / sqrt(b2) : 0.0;
      in.seconds = c->wall_khz > 0.0 ? (double)(sr.t1 - sr.t0) / (c->wall_khz * 1e3) : 0.0;
    }
    for (const auto& pt : run.parts) e->free_lanes.push_back(pt.lane);
    hooks.done(jb.tag, any_fail ? HZ_WARN_NOCONV : HZ_OK, info);
    return HZ_OK;
  };
  // A new job: its model, ceil(nrhs / width) lanes per frequency (the lanes
  // of one frequency share the first one's tables), its right-hand sides started.
  auto admit = [&](EngineJob& jb) -> int {
    hz_engine::Running run;
    run.job = jb;
    const int per = (jb.nrhs + W - 1) / W;
    for (int fi = 0; fi < jb.nfreq; ++fi)
      for (int q = 0; q < per; ++q) {
        run.parts.push_back({e->free_lanes.back(), fi, q * W, std::min(W, jb.nrhs - q * W)});
        e->free_lanes.pop_back();
      }
    const int model = run.parts[0].lane;
    double mmin = 0.0, mmax = 0.0;
    int rc = engine_model(e, model, jb.m_dev, &mmin, &mmax);
    std::vector<int> sl;
    int first = -1;
    for (const auto& pt : run.parts) {
      if (rc) break;
      if (pt.off == 0) {
        first = pt.lane;
        rc = engine_lane_setup(e, pt.lane, model, mmin, mmax, jb.freq_hz[pt.fi], jb.alpha);
        if (rc) break;
      } else {
        e->ft[pt.lane] = e->ft[first];
        HZ_HIP(c, hipMemcpyAsync(c->freqtab.as<FreqTab>() + pt.lane, &e->ft[pt.lane], sizeof(FreqTab),
                                 hipMemcpyHostToDevice, st));
      }
      std::vector<Slot> srec(pt.cnt);
      for (int k = 0; k < pt.cnt; ++k) {
        memset(&srec[k], 0, sizeof(Slot));
        srec[k].status = kActive;
        srec[k].freq = pt.lane;
        srec[k].rh_nnz = -1;
        sl.push_back(pt.lane * W + k);
      }
      HZ_HIP(c, hipMemcpyAsync(bt.slots + pt.lane * W, srec.data(), pt.cnt * sizeof(Slot), hipMemcpyHostToDevice, st));
      HZ_HIP(c, hipMemcpyAsync(Bv + (size_t)pt.lane * W * n0, jb.b_dev + ((size_t)pt.fi * jb.nrhs + pt.off) * n0,
                               (size_t)pt.cnt * n0 * sizeof(double2), hipMemcpyDeviceToDevice, st));
      HZ_HIP(c, hipStreamSynchronize(st));  // srec is read before it goes out of scope
    }
    if (rc != HZ_OK) {
      for (const auto& pt : run.parts) e->free_lanes.push_back(pt.lane);
      std::vector<hz_rhs_info> none;
      hooks.done(jb.tag, rc, none);
      return HZ_OK;  // the job is refused; the engine goes on
    }
    Batch lb;
    if ((rc = engine_list(e, sl, &lb)) != HZ_OK) return rc;
    HZ_HIP(c, it.start(lb, (int)sl.size(), Bv, 0, 0));
    for (const auto& pt : run.parts)
      HZ_HIP(c, launch_rh_sparse(n0, pt.cnt, bt, Bv, c->rh_idx.as<int>(), c->rh_val.as<double2>(), n0, st,
                                 pt.lane * W));
    e->running.push_back(std::move(run));
    return HZ_OK;
  };

  int cap = 0;
  long long iters_issued = 0;
  int rc = HZ_OK;
  for (;;) {
    // summaries of finished units
    while (!pending.empty() && ((int)pending.size() > kLag || cap == 0)) {
      const auto [useq, k] = pending.front();
      pending.pop_front();
      HZ_HIP(c, hipEventSynchronize(c->ev[k]));
      const Summary sm = c->ring_host[k];
      if (restart_seq > useq) continue;
      const bool fresh = admit_seq < useq;  // every running job's slots were in this unit's list
      if (sm.nrestart > 0) {
        HZ_HIP(c, it.restart(nslots));
        restart_seq = seq;
        if ((rc = close_unit()) != HZ_OK) return rc;
        cap = nslots;
        continue;
      }
      if (!fresh) continue;
      cap = std::min(cap, sm.nactive);
      it.dense_rh = sm.ndense > 0;
      const int* fs = e->fst_host + (size_t)k * (e->lanes + 1);
      for (size_t j = 0; j < e->running.size();) {
        bool all_done = true;
        for (const auto& pt : e->running[j].parts) all_done = all_done && fs[pt.lane + 1] == fs[pt.lane];
        if (!all_done) {
          ++j;
          continue;
        }
        if ((rc = finish(e->running[j])) != HZ_OK) return rc;
        e->running.erase(e->running.begin() + j);
      }
    }
    // New jobs between iterations, after an even number of them: a slot's
    // first iteration is then a ring-0 one, as in hz_solve, so its iterate
    // is advanced in the same order and comes out bitwise the same. With no
    // job left every pending term has been flushed and the count restarts.
    if (e->running.empty()) iters_issued = 0;
    const bool idle = e->running.empty() && pending.empty();
    std::vector<EngineJob> jobs;
    bool go = true;
    if ((iters_issued & 1) == 0) go = hooks.next((int)e->free_lanes.size(), idle, jobs);
    int added = 0;
    for (EngineJob& jb : jobs) {
      if (jb.nrhs < 1 || jb.nfreq < 1 || (long long)jb.nfreq * ((jb.nrhs + W - 1) / W) > (long long)e->free_lanes.size()) {
        std::vector<hz_rhs_info> none;
        hooks.done(jb.tag, HZ_ERR_ARG, none);
        continue;
      }
      if ((rc = admit(jb)) != HZ_OK) return rc;
      added += jb.nfreq * jb.nrhs;
    }
    if (added > 0) {
      admit_seq = seq;
      it.dense_rh = true;  // until a summary has seen the new slots' lists
      cap = std::min(nslots, cap + added);
      if ((rc = close_unit()) != HZ_OK) return rc;
    }
    if (!go && e->running.empty() && pending.empty()) break;
    if (cap == 0) {
      // nothing to iterate: take a summary so that finished jobs are seen
      if (pending.empty() && !e->running.empty() && (rc = close_unit()) != HZ_OK) return rc;
      continue;
    }
    HZ_HIP(c, it.issue(cap, st, (int)(iters_issued & 1)));
    ++iters_issued;
    if ((rc = close_unit()) != HZ_OK) return rc;
  }
  HZ_HIP(c, hipStreamSynchronize(st));
  return HZ_OK;
}

}  // namespace hz
