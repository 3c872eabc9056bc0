// Internal declarations shared by the HIP kernels and the C-ABI host code.
// Everything here is complex128 (double2 = interleaved re, im) and FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hz.h"

namespace hz {

constexpr int kMaxLevels = 12;
constexpr int kBlock = 256;        // threads per block of the grid kernels
constexpr int kVecPerThread = 4;   // nodes per thread in the pointwise Krylov kernels
constexpr int kCoarseWaves = 4;    // waves per block of the coarse solve (each its own 16-row tile)
constexpr int kPcrMax = 2048;      // longest 1D grid for the exact tridiagonal solve
// Most unknowns on a coarsest level that is solved exactly. The dense inverse
// takes one Gauss-Jordan launch per pivot over an (n x n) complex matrix per
// frequency, so its set-up grows as n^3: 4096 unknowns is 268 MB per frequency
// and well under a second; larger coarsest levels are refused.
constexpr int kCoarseMax = HZ_COARSE_MAX;

// Per right-hand-side solver status. Finished states equal the HZ_RHS_* codes.
enum : int {
  kActive = -1,
  kConverged = 0,
  kMaxit = 1,
  kBreakdown = 2,
  kNonfinite = 3,
  kRestart = 4,  // breakdown seen; waits for the one restart with rhat = r
};

// One multigrid level's grid: node counts, spacing and injected slowness.
struct Grid {
  int nz, nx;
  double h;
  const double* m;  // device, [nz][nx] ([nz][ny][nx] on 3D grids)
  int ny = 1;       // 3D grids only
  // models of several requests in one batch: frequency entry f reads its
  // slowness at m + FreqTab::model * mstride (0: one model for every entry)
  size_t mstride = 0;
  // density of Eq. (1) on this level, [nz][nx] ([nz][ny][nx] on 3D grids;
  // null: constant density, the operator of Eq. (2))
  const double* rho = nullptr;
  // 2D grids with a density: the level's coupling table (RhoC in hz_device.h),
  // [3][nz][nx]; the fused kernels read it instead of rho
  const double* dc = nullptr;
  // 2D finest level of the fused BiCGSTAB path: the row pitch of the level's
  // vectors, > nx so that every row starts on a 128-byte line (0: nx). The
  // tables above stay [nz][nx]. Only the kernels of that path read it.
  int px = 0;
};

// the row pitch of a 2D level's vectors
__host__ __device__ inline int vpitch(const Grid& g) { return g.px > 0 ? g.px : g.nx; }

// The row pitch of the finest level's vectors on the fused 2D BiCGSTAB path:
// nx rounded up to 8 complex values (128 bytes), and the nodes per slot the
// finest-level vector buffers hold (the pitched rows on 2D grids).
inline int fine_pitch(int nx) { return (nx + 7) & ~7; }
inline size_t fine_nodes(int dim, int nz, int ny, int nx) {
  return dim == 2 ? (size_t)nz * fine_pitch(nx) : (size_t)nz * ny * nx;
}

// Per-frequency constants (device table).
struct FreqTab {
  double omega;
  double sB_re, sB_im;  // mass shift of B: 1 - j alpha
  double sM_re, sM_im;  // mass shift of M: beta1 - j beta2
  double wj[kMaxLevels];
  const double2* cinv;               // inverse of M on the coarsest level, [nc][nc]
  int coarse_jacobi;                 // 1: the coarsest level is smoothed, not solved exactly
  const double2* winv[kMaxLevels];   // w_l / diag(M_l) on each smoothing level, [n_l]
  int model;                         // which model of the batch (see Grid::mstride)
};

// Per right-hand-side Krylov scalars (device array, one per slot).
struct Slot {
  double2 rho, alpha, omega, beta;
  double bnorm2, rnorm2;
  int iters, status, restarted, freq;
  unsigned long long t0, t1;  // device wall clock at the start and at the last iteration
  int phase;                  // GMRES: 0 = Arnoldi steps, 1 = cycle end pending
  int cyc_k;                  // GMRES: Arnoldi steps taken in the current cycle
  double2 scal;               // GMRES: divisor of the newest basis vector (real part)
  int rh_nnz;                 // BiCGSTAB: nonzeros of the shadow residual r^ held in the sparse
                              // list (Batch::rh_idx/rh_val), -1: r^ is used as a dense vector
  int pending;                // BiCGSTAB: pend_alpha ph0 + pend_omega sh0 not yet added to x
  double2 pend_alpha, pend_omega;
};

// A shadow residual r^ = b with at most this many nonzeros (point sources,
// receiver sets) is also kept as a list, and the inner products with it are
// formed from the list instead of streaming r^.
constexpr int kShadowMax = 256;

// Complex vectors per right-hand side on the finest grid (r, r^, two p
// buffers, v, two p^ buffers, s, two s^ buffers, t and two smoothing buffers).
constexpr int kFineVectors = 13;

// GMRES(m) per-slot small arrays (device): the Hessenberg matrix column-major
// H[slot][j*(m+1) + i] (rotated) and Hu (as the Arnoldi process forms it),
// right-hand side g, rotations (cs, sn), solution y and the current step's two
// coefficient vectors (the second pass's s and the update's c).
struct Gmres {
  double2* H;        // Hessenberg matrix after the Givens rotations, [slots][m][m+1] (column-major)
  double2* Hu;       // the Arnoldi coefficients themselves, the same layout
  double2* g;
  double* cs;
  double2* sn;
  double2* y;
  double2* hc;       // [slots][2][m+1]: a step's coefficients s and c (k_gm_fin2)
  double* partials;  // [slots][max_tiles][width]
  int m;
  int max_tiles;
  int width;         // doubles per tile of the partials, 4 (m + 1) + 4
};

// The batch every kernel works on: the compacted list of active slots.
struct Batch {
  const int* active;   // [capacity] slot ids, valid up to *nactive
  const int* nactive;  // device count
  Slot* slots;
  const FreqTab* ft;
  const int* fstart;   // [nfreq + 1]: the list's entries of frequency f are fstart[f]..fstart[f+1]-1
  const int* rh_idx;      // [capacity][kShadowMax] node indices of r^'s nonzeros, ascending
  const double2* rh_val;  // [capacity][kShadowMax] their values
};

// Scratch for deterministic per-slot reductions: block partial sums.
constexpr int kPartialWidth = 4;
struct Reduce {
  double* partials;  // [slots][max_tiles][kPartialWidth]
  int max_tiles;
};

// Summary the host polls: counts of active and restart-pending slots.
struct Summary {
  int nactive, nrestart, nother;  // nother: active slots in the other GMRES phase
  int ndense;                     // active slots whose shadow residual r^ is a dense vector
};

struct Tiles {
  int tx, tz;     // block shape (tx * tz == kBlock)
  int ntx, ntz;   // tiles per axis
  int per_slot;   // ntx * ntz
};

Tiles grid_tiles(int nz, int nx, int dim);
int vec_tiles(size_t n);
// Level hierarchy (hz_api.hip): an axis of n nodes halves to ceil(n / 2).
int coarse_n(int n);
int grid_max_levels(int dim, int nz, int nx);      // most levels the grid allows
int grid_default_levels(int dim, int nz, int nx);  // levels of a default plan
long long tile_blocks(int per_slot, int cap);  // XCD-aware grid size of a 2D-tiled kernel
int lds_tiles(int nz, int nx);                 // tiles per slot of the LDS-staged 2D kernels
// tiles per slot of the kernels that store reduction partials over a grid
int reduce_tiles(int nz, int nx, int dim);

// The small levels of a 2D V-cycle, walked by one workgroup per right-hand
// side (hz_vsmall.hip): smoothing levels l0 .. L-2 and the coarsest level
// L-1. Arrays are indexed by level; n is each level's slot stride.
// Most nodes of a level the fused kernels take: one complex vector of the
// largest such level is held in LDS (96 KB).
constexpr int kSmallNodes = 6144;
struct SmallLevels {
  int l0, L;
  int coarse_sweeps;  // sweeps on the coarsest level of frequencies that smooth it (0: none)
  double coarse_w;    // their damped-Jacobi weight
  Grid g[kMaxLevels];
  double2* b[kMaxLevels];  // right-hand sides (b[l0] is the input)
  double2* u[kMaxLevels];  // V-cycle results (u[l0] is the output; u[L-1] the coarse solution)
  double2* x[kMaxLevels];  // pre-smoothed iterate, kept for the ascent; work vector on the coarsest level
  double2* y[kMaxLevels];  // residual, then u2 + P e
  size_t n[kMaxLevels];
};
// Descent (to the coarse right-hand side, and the coarsest level's sweeps for
// frequencies that smooth it) and ascent, one workgroup per entry of the
// active list (cap entries at most).
size_t small_levels_lds(const SmallLevels& s);  // LDS bytes per workgroup of the two kernels
hipError_t launch_vdown(const SmallLevels& s, const Batch& bt, int cap, hipStream_t st);
hipError_t launch_vup(const SmallLevels& s, const Batch& bt, int cap, hipStream_t st);

// ---- kernel launchers (hz_kernels.hip) ----------------------------------------
// All take the stream last and return the launch status.
// `which` selects the mass shift: 0 = B (1 - j alpha), 1 = M (beta1 - j beta2).

hipError_t launch_apply(int dim, const Grid& g, int lvl, int which, const Batch& bt, int cap,
                        const double2* x, double2* y, size_t stride, hipStream_t st);
hipError_t launch_smooth(int dim, const Grid& g, int lvl, double w_override, const Batch& bt,
                         int cap, const double2* b, const double2* u_in, double2* u_out,
                         size_t stride, hipStream_t st);
// 3D: one marching sweep from u_in, or (from_zero, u_in unused) two sweeps from
// u = 0, or (e given) one sweep from u_in + P e with e on the coarser level gc
// (slot stride sc); constant density only
hipError_t launch_march3(const Grid& g, int lvl, const Batch& bt, int cap, bool from_zero, const double2* b,
                         const double2* u_in, double2* u_out, size_t stride, hipStream_t st,
                         const Grid* gc = nullptr, const double2* e = nullptr, size_t sc = 0);
// 3D, constant density: u_out = two sweeps from u_in + P e (e on the coarser
// level gc, slot stride sc) in one march; u_out must not be u_in
hipError_t launch_post3(const Grid& g, const Grid& gc, int lvl, const Batch& bt, int cap, const double2* b,
                        const double2* u_in, const double2* e, double2* u_out, size_t stride, size_t sc,
                        hipStream_t st);
hipError_t launch_restrict(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                           const double2* b, const double2* u, double2* bc, size_t sf,
                           size_t sc, hipStream_t st);
// The same restriction with the fine residual b - M u first stored in
// scratch (a fine-level vector, 3D grids; other dimensions ignore it).
hipError_t launch_restrict_via(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                               const double2* b, const double2* u, double2* scratch, double2* bc, size_t sf,
                               size_t sc, hipStream_t st);
hipError_t launch_prolong(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                          const double2* e, const double2* u_in, double2* u_out, size_t sf,
                          size_t sc, hipStream_t st);
// 1D grids: mode 0: b given (in_a); 1: b = p = in_a + beta (in_b - omega in_c)
// stored to bout; 2: b = s = in_a - alpha in_b stored to bout. u2 = two
// Jacobi sweeps from zero. (2D grids use launch_pre2r.)
hipError_t launch_pre2(int dim, const Grid& g, int lvl, int mode, const Batch& bt, int cap,
                       const double2* in_a, const double2* in_b, const double2* in_c, double2* bout,
                       double2* u2, size_t stride, hipStream_t st);
// u_out = S(u2 + P e): prolongation, correction and one sweep.
hipError_t launch_prolong_smooth(int dim, const Grid& gf, const Grid& gc, int lvl, const Batch& bt,
                                 int cap, const double2* e, const double2* b, const double2* u2,
                                 double2* u_out, size_t sf, size_t sc, hipStream_t st);
// 2D only: two damped-Jacobi sweeps from zero (u2) on the right-hand side
// formed as in launch_pre2 (stored to bout in modes 1/2), and the
// full-weighting restriction of the residual b - M u2 stored to bcoarse; u2
// itself is stored only when u2 is not null
// chunk_rows: grid rows per wavefront (even); any even value gives the same
// result, the fastest one depends on the level and the batch size.
hipError_t launch_pre2r(const Grid& g, const Grid& gc, int lvl, int mode, const Batch& bt, int cap,
                        const double2* a, const double2* b, const double2* c, double2* bout, double2* u2,
                        double2* bcoarse, size_t stride, size_t sc, int chunk_rows, hipStream_t st);
// 2D only: u_out = two damped-Jacobi sweeps on M from u2 + P e, with u2 the
// two pre-sweeps from zero on b formed again (as launch_pre2r forms them)
hipError_t launch_post2(const Grid& gf, const Grid& gc, int lvl, const Batch& bt, int cap, const double2* e,
                        const double2* b, double2* u_out, size_t sf, size_t sc, int chunk_rows, hipStream_t st);
// u_out = `sweeps` damped-Jacobi sweeps (weight w) from zero on level lvl, for
// the slots whose frequency has coarse_jacobi set; tmp is a work vector
hipError_t launch_coarse_jacobi(int dim, const Grid& g, int lvl, double w, int sweeps, const Batch& bt, int cap,
                                const double2* b, double2* tmp, double2* u_out, size_t stride, hipStream_t st);
hipError_t launch_coarse_solve(int nc, int nfreq, int nrhs, const Batch& bt, const double2* bc,
                               double2* uc, size_t stride, hipStream_t st);
hipError_t launch_pcr(const Grid& g, const Batch& bt, int cap, const double2* b, double2* u,
                      size_t stride, hipStream_t st);
// winv[p] = w / diag(M)[p] on one level for one frequency.
hipError_t launch_winv(int dim, const Grid& g, double omega, double s_re, double s_im, double w,
                       double2* winv, hipStream_t st);

// Gauss-Jordan inversion of the coarsest M for nfreq frequencies.
hipError_t launch_assemble_dense(int dim, const Grid& g, int nfreq, const FreqTab* ft,
                                 double2* A, hipStream_t st);
hipError_t launch_gj_step(int nc, int nfreq, int k, const double2* A_in, double2* A_out,
                          hipStream_t st);

// BiCGSTAB pieces. Each producer stores block partials; launch_bicg_fin
// (one block per slot) sums them in a fixed order and updates the slot's
// scalars and status.
// (v null in init and restart: v is not stored). Init and restart take n
// nodes in [nz][nx] order: px > 0 places node i of row i / nx at
// (i / nx) * px + i % nx in x, r, rh, p and v (rows of pitch px; b keeps
// [nz][nx] rows, slot stride bstride, 0: stride); their sums then group as
// with px = 0.
hipError_t launch_bicg_init(size_t n, const Batch& bt, int cap, const Reduce& rd,
                            const double2* b, double2* x, double2* r, double2* rh, double2* p,
                            double2* v, size_t stride, hipStream_t st, size_t bstride = 0, int nx = 0,
                            int px = 0);
hipError_t launch_bicg_p(size_t n, const Batch& bt, int cap, const double2* r, const double2* p_old,
                         const double2* v, double2* p_new, size_t stride, hipStream_t st);
// v null (2D only): no store; only the slots whose r^ is dense get a partial.
hipError_t launch_bicg_apply_sigma(int dim, const Grid& g, const Batch& bt, int cap,
                                   const Reduce& rd, const double2* ph, const double2* rh,
                                   double2* v, size_t stride, hipStream_t st);
hipError_t launch_bicg_s(size_t n, const Batch& bt, int cap, const double2* r, const double2* v,
                         double2* s, size_t stride, hipStream_t st);
// t null (2D only): no store, only the partials <t, s>, <t, t>.
hipError_t launch_bicg_apply_omega(int dim, const Grid& g, const Batch& bt, int cap,
                                   const Reduce& rd, const double2* sh, const double2* s,
                                   double2* t, size_t stride, hipStream_t st);
// ring -1: x += alpha ph + omega sh; ring 0: x unchanged, the term left
// pending (recorded by the step reduction); ring 1: x += pending term (ph0,
// sh0: ring 0's buffers) + alpha ph + omega sh.
hipError_t launch_bicg_xr(size_t n, const Batch& bt, int cap, const Reduce& rd, double2* x,
                          const double2* ph, const double2* sh, const double2* s, const double2* t,
                          double2* r, const double2* rh, size_t stride, hipStream_t st, int ring = -1,
                          const double2* ph0 = nullptr, const double2* sh0 = nullptr);
// The same update on a 2D grid with t = B sh formed from sh (no stored t; the
// partials per LDS tile, reduce_tiles(nz, nx, 2) of them per slot).
hipError_t launch_bicg_xr_t(const Grid& g, const Batch& bt, int cap, const Reduce& rd, double2* x,
                            const double2* ph, const double2* sh, const double2* s, double2* r,
                            const double2* rh, size_t stride, hipStream_t st, int ring, const double2* ph0,
                            const double2* sh0);
// Adds the pending term to x (all nslots slots, or only those about to restart).
// (slots slot0 .. slot0 + nslots - 1)
hipError_t launch_bicg_flush(size_t n, int nslots, const Batch& bt, int only_restart, double2* x,
                             const double2* ph0, const double2* sh0, size_t stride, hipStream_t st, int slot0 = 0);
hipError_t launch_bicg_restart(size_t n, int nslots, const Batch& bt, const Reduce& rd,
                               const double2* r, double2* rh, double2* p, double2* v,
                               size_t stride, hipStream_t st, int nx = 0, int px = 0);
// The sparse list of r^ = b for every one of the nslots slots (rh_nnz = -1
// where b has more than kShadowMax nonzeros). idx/val: the arrays Batch
// points to, writable.
hipError_t launch_rh_sparse(size_t n, int nslots, const Batch& bt, const double2* b, int* idx, double2* val,
                            size_t stride, hipStream_t st, int slot0 = 0);
enum : int { kFinInit = 0, kFinSigma = 1, kFinOmega = 2, kFinStep = 3, kFinRestart = 4, kFinSigmaB = 5 };
// tiles: the producer's tiles per slot; restart runs over all nslots slots.
// vec: for sigma v, for sigma-B p^ (v = B p^ is formed at the nodes of a
// sparse r^; g: the finest 2D grid), for step r (the inner products with a
// sparse r^ are formed here from it); unused otherwise.
// ring (step only): 0 records the update's term as pending, 1 clears it.
// restart_at (step only, > 0): take the restart after that many iterations.
hipError_t launch_bicg_fin(int which, int tiles, const Batch& bt, int cap, const Reduce& rd,
                           double tol, int maxit, const double2* vec, size_t stride, hipStream_t st,
                           int ring = -1, int restart_at = 0, const Grid* g = nullptr);
hipError_t launch_compact(int nslots, int nrhs, int nfreq, Slot* slots, int* active, int* nactive,
                          int* fstart, Summary* sum, int want_phase, hipStream_t st);
hipError_t launch_copy(const Batch& bt, int cap, size_t n, const double2* x, double2* y,
                       size_t stride, hipStream_t st);
// dst = src for nslots slots of an nz x nx grid, rows of pitch sp in src
// (slot stride ss) and dp in dst (slot stride ds); dst's padding is zeroed
hipError_t launch_repitch(int nslots, int nz, int nx, const double2* src, int sp, size_t ss, double2* dst, int dp,
                          size_t ds, hipStream_t st);

// ||b - B x||^2 and ||b||^2 per slot of the list into out[slot*2 + {0,1}]
hipError_t launch_true_residual(int dim, const Grid& g, const Batch& bt, int cap,
                                const Reduce& rd, const double2* b, const double2* x,
                                double* out, size_t stride, hipStream_t st);

// GMRES pieces
hipError_t launch_gm_residual(int dim, const Grid& g, const Batch& bt, int cap, const Reduce& rd,
                              const Gmres& gm, int first, double tol, int maxit, const double2* b,
                              double2* x, double2* v0, size_t stride, hipStream_t st);
hipError_t launch_gm_scale(size_t n, const Batch& bt, int cap, double2* v, size_t stride,
                           hipStream_t st);
// One Arnoldi step j of GMRES (k_gm_dots2, k_gm_fin2, k_gm_update2 in
// hz_krylov.hip) for u_j = V_j and z = B M^-1 u_j; finish (z null): the pass
// that completes the cycle's last column only.
int gm_dot_tiles(size_t n);  // tiles of GMRES's dot pass over n nodes (partials per slot)
hipError_t launch_gm_step(size_t n, const Batch& bt, int cap, const Gmres& gm, int j, int finish, double tol,
                          int maxit, double2* V, size_t vstride, const double2* z, size_t stride, hipStream_t st);
hipError_t launch_gm_solve(const Batch& bt, int cap, const Gmres& gm, hipStream_t st);
hipError_t launch_gm_combine(size_t n, const Batch& bt, int cap, const Gmres& gm,
                             const double2* V, size_t vstride, double2* t, size_t stride,
                             hipStream_t st);
hipError_t launch_axpy1(size_t n, const Batch& bt, int cap, const double2* z, double2* x,
                        size_t stride, hipStream_t st);

// misfit helpers
hipError_t launch_point_rhs(size_t n, int nsrc, const int* nodes, const double2* amp,
                            double scale, double2* b, hipStream_t st);
hipError_t launch_gather(int nrhs, int nrec, const int* rec_nodes, const double2* u,
                         size_t stride, double2* d, hipStream_t st);
hipError_t launch_misfit(size_t nd, const double2* d_obs, const double2* d_cal, size_t nm,
                         const double* m, double lambda, double* out, hipStream_t st);
hipError_t launch_inject(const Grid& gf, int dim, double* mc, hipStream_t st);

// FWI gradient pieces (hz_fwi.hip)
hipError_t launch_adjoint_src(int nslots, size_t n, int nuniq, const int* uniq_node, const int* rec_ptr,
                              const int* rec_idx, int nrec, const double2* u, const double2* d_obs,
                              double2* out, hipStream_t st);
hipError_t launch_grad_accum(int dim, const Grid& g, int nfreq, int nsrc, const double* omega, double alpha,
                             const double2* u, const double2* mu, double lambda, const double* reg,
                             int accumulate, double* grad, hipStream_t st);
hipError_t launch_born_src(int dim, const Grid& g, int nslots, int nsrc, const double* omega, double alpha,
                           const double2* u, const double* v, double2* rhs, hipStream_t st);
hipError_t launch_adjoint_data(int nslots, size_t n, int nuniq, const int* uniq_node, const int* rec_ptr,
                               const int* rec_idx, int nrec, const double2* y, double2* out, hipStream_t st);
hipError_t launch_cg(int mode, size_t n, const double* g, const double* Hp, double* x, double* r, double* p,
                     double* state, double tol, hipStream_t st);
hipError_t launch_check_model(size_t n, const double* m, double* out3, hipStream_t st);
// The coupling table of a 2D level with a density (Grid::dc) from g.rho.
hipError_t launch_density_coef(const Grid& g, double* dc, hipStream_t st);
// out3 = {min m / sqrt(rho), max m / sqrt(rho), count of rho entries that are
// not finite and positive} (the extremes over the valid entries)
hipError_t launch_check_density(size_t n, const double* m, const double* rho, double* out3, hipStream_t st);

}  // namespace hz
