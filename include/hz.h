/*
 * hz.h -- C ABI of the MI355X (gfx950) shifted-Laplace preconditioned
 * Helmholtz solver.
 *
 * Problem (Kazemi, arXiv:1712.08743, section "Full waveform inversion in the
 * space-frequency domain"): given the real slowness model m = 1/c, the
 * angular frequency omega = 2 pi f, the damping alpha and sources f, solve
 * the discretised constant-density Helmholtz equation of Eq. (2)-(3),
 *     B u = f,   B = -Laplace_h - omega^2 m^2 (1 - j alpha),
 * with a first-order absorbing boundary (Eq. (1)), and evaluate the misfit
 * J(m) of Eq. (4) at the receivers. The solve is a right-preconditioned
 * Krylov method (BiCGSTAB, or GMRES(m) as in the paper's own data-modelling
 * engine) whose preconditioner is the shifted Laplacian
 *     M = -Laplace_h - (beta1 - j beta2) omega^2 m^2
 * applied approximately by one geometric multigrid V-cycle.
 *
 * Discretisation (the paper leaves it open; this library's reading):
 *   nodes (iz, ix), z = iz h, x = ix h, flat index iz*nx + ix, z = 0 is the
 *   surface; every edge absorbs with du/dn + j omega m u = 0; centred second
 *   differences with the ghost node eliminated; rows scaled by the control
 *   volume weight (1/2 per axis on end nodes), so that
 *     B = L/h^2 + (j omega/h) diag(g m) - omega^2 (1 - j alpha) diag(w m^2)
 *   is complex symmetric. Right-hand sides are in this weighted form: a unit
 *   point source at node p is b = e_p / h^dim.
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device memory on the context's device; the
 *     others are host memory. The caller owns all of them; the library never
 *     keeps a caller pointer after a call returns.
 *   - Complex values are interleaved (re, im) doubles: hz_c128 has the layout
 *     of C99 double _Complex and of a torch.complex128 element.
 *   - Vectors are stored [rhs][nz][nx] with x fastest (1D: [rhs][n]).
 *   - All device work is ordered on the stream given to hz_create; each call
 *     returns after that work has completed.
 *   - A context is not thread-safe; use one context per host thread/stream.
 *   - Return value: HZ_OK (0), a positive warning, or a negative error. No
 *     exception crosses the ABI. hz_last_error() describes the last failure.
 */
#ifndef HZ_H
#define HZ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hz_c128;

typedef struct hz_ctx hz_ctx;

/* return codes */
#define HZ_OK            0
#define HZ_WARN_NOCONV   1   /* output written; some right-hand side did not converge */
#define HZ_ERR_ARG      -1   /* null pointer, bad size or value, non-finite or non-positive slowness */
#define HZ_ERR_SHAPE    -2   /* grid cannot be coarsened to the requested level count, or the
                                coarsest level is solved exactly and has more than
                                HZ_COARSE_MAX unknowns */
#define HZ_COARSE_MAX 4096   /* most unknowns of an exactly solved coarsest level (its dense
                                inverse costs n^3 work and 16 n^2 bytes per frequency) */
#define HZ_ERR_NOMEM    -3   /* device allocation failed or workspace budget exceeded */
#define HZ_ERR_DEVICE   -4   /* a HIP runtime error */
#define HZ_ERR_STATE    -5   /* no model set */

/* Krylov method */
#define HZ_BICGSTAB      0
#define HZ_GMRES         1

/* preconditioner */
#define HZ_PRECOND_MG    0   /* one V-cycle approximating M^-1 */
#define HZ_PRECOND_EXACT 1   /* exact M^-1 (1D only: tridiagonal solve) */
#define HZ_PRECOND_NONE  2

/* solve on the coarsest multigrid level */
#define HZ_COARSE_AUTO   0   /* exact, unless the level's smallest kh = omega h_c m_min is >= 2.5,
                                where damped Jacobi converges for every mode (local Fourier
                                analysis): then coarse_sweeps sweeps */
#define HZ_COARSE_EXACT  1   /* dense inverse of M on that level, per frequency */
#define HZ_COARSE_JACOBI 2   /* coarse_sweeps damped-Jacobi sweeps (weight 0.8) from zero */

/* per right-hand-side status */
#define HZ_RHS_CONVERGED 0
#define HZ_RHS_MAXIT     1
#define HZ_RHS_BREAKDOWN 2
#define HZ_RHS_NONFINITE 3

#define HZ_MAX_LEVELS   12

typedef struct {
    int    device;                  /* HIP device ordinal */
    void  *hip_stream;              /* hipStream_t to order work on; NULL = the null stream */
    size_t workspace_budget_bytes;  /* 0 = no limit beyond the device's memory */
} hz_ctx_opts;

typedef struct {
    int    krylov;          /* HZ_BICGSTAB (default) or HZ_GMRES */
    int    gmres_m;         /* GMRES restart length (default 30, at most 200) */
    double tol;             /* stop when ||b - B u|| <= tol ||b|| (default 1e-8) */
    int    maxit;           /* iteration cap per right-hand side (default 10000) */
    int    precond;         /* HZ_PRECOND_* (default HZ_PRECOND_MG) */
    double beta1, beta2;    /* shift of M (default 1, 0.5); beta2 must be > 0 */
    int    levels;          /* V-cycle levels incl. the finest; 0 = halve (an axis of n nodes to
                               ceil(n/2)) until the coarsest level has at most 512 unknowns */
    int    nu1, nu2;        /* pre- and post-smoothing sweeps (default 2, 2) */
    double jacobi_w;        /* largest damped-Jacobi weight the plan may use (default 0.8) */
    const double *jacobi_w_level; /* host, optional: fixed weight per smoothing level
                                     (levels-1 values, every frequency); NULL = plan by LFA */
    int    autotune;        /* 1 (default): the first launch of a fused V-cycle kernel for a
                               (kernel, level grid, batch-size octave) times the candidate
                               launch shapes and keeps the fastest for the context; 0: a
                               fixed shape. Results do not depend on the shape. */
    int    chunk_rows;      /* 0 (default): shape from the tuner (or fixed); > 0, even: grid
                               rows per wavefront for every fused V-cycle kernel */
    int    coarse;          /* HZ_COARSE_* (default HZ_COARSE_AUTO) */
    int    coarse_sweeps;   /* sweeps where the coarsest level is smoothed (default 2, 1..64) */
    int    graphs;          /* 1: BiCGSTAB iterations are captured in HIP graphs (two
                               iterations per graph, one graph per batch-size bucket) and
                               replayed; 0 (default): every launch issued one by one. Ignored
                               while kernel timing is on. Results do not depend on it. */
    int    restart_at;      /* for tests of the breakdown path: > 0 makes every BiCGSTAB
                               right-hand side take the one restart (r^ = r, p = v = 0) after
                               this many iterations, as after a breakdown; 0 (default): off */
    int    plain;           /* 1: the plain per-launch path, kept as a point of comparison:
                               every step of the iteration is a kernel of its own (single
                               smoothing sweeps, residual and restriction, prolongation, operator
                               apply and vector updates), the shadow residual is a dense vector,
                               the iterate is advanced every iteration, and the host reads each
                               iteration's scalars back before it issues the next. Same
                               iteration, results agree to rounding. 0 (default): the fused
                               batched path. */
} hz_solve_opts;

typedef struct {
    int    status;          /* HZ_RHS_* */
    int    iters;           /* Krylov iterations (BiCGSTAB: two preconditioner and two
                               operator applications each; GMRES: one of each) */
    double relres;          /* true ||b - B u|| / ||b|| of the returned u (0 if b = 0) */
    double seconds;         /* device time from the start of the solve to this right-hand
                               side's last iteration (device wall clock) */
} hz_rhs_info;

/* Fill *o with the defaults listed above. */
void hz_default_opts(hz_solve_opts *o);

/* Create a context on a device and stream. *out receives the context.
 * Errors: HZ_ERR_ARG (null out or o, bad device), HZ_ERR_DEVICE. */
int  hz_create(hz_ctx **out, const hz_ctx_opts *o);

/* Release every device buffer of the context. NULL is allowed. */
void hz_destroy(hz_ctx *c);

/* Set the slowness model m (Eq. (2): m = 1/c, real, s/m), dim 1 or 2.
 * dim 1: nz must be 1 and nx >= 3 is the node count. dim 2: nz, nx >= 3.
 * m_dev: device, [nz][nx] doubles, copied (the caller may free it after).
 * Builds the injected slowness of every coarser level.
 * Errors: HZ_ERR_ARG (bad sizes, h <= 0, non-finite or non-positive m). */
int  hz_set_model(hz_ctx *c, int dim, int nz, int nx, double h, const double *m_dev);

/* Variable density (Eq. (1): -div(rho grad u) - k^2 (1 - j alpha) u = f) on
 * the model set last (1D, 2D or 3D). rho_dev: device, [nz][nx] doubles
 * ([nz][ny][nx] in 3D), finite and positive, copied; NULL returns to
 * constant density (Eq. (2)). A new hz_set_model or hz_set_model_3d also
 * does. Discretisation: the coupling of two neighbouring
 * nodes is multiplied by the mean (rho_p + rho_q) / 2 of their densities,
 * and the absorbing boundary is written for the flux, rho du/dn + j omega m
 * sqrt(rho) u = 0, so its term carries sqrt(rho_p); the shifted Laplacian M
 * takes the same couplings and boundary term. The density is injected to
 * the coarse levels like the slowness, and the V-cycle is planned for the
 * slowness m / sqrt(rho) the equation propagates with. Every call on the
 * model (hz_solve, hz_solve_noalloc, hz_precond, hz_apply, hz_smooth,
 * hz_restrict, the misfit, gradient and Gauss-Newton calls, whose dB/dm
 * carries sqrt(rho) in its boundary part) then uses the density. On 2D
 * grids the fused kernels read a per-level table of the couplings (three
 * doubles per node of every level, built here: about 32 bytes per fine
 * node in all); 1D and 3D grids take the one-kernel-per-step V-cycle. The
 * serving calls are not affected.
 * Errors: HZ_ERR_ARG (no model, non-finite or non-positive rho),
 * HZ_ERR_NOMEM, HZ_ERR_DEVICE. */
int  hz_set_density(hz_ctx *c, const double *rho_dev);

/* Point sources in weighted form: b_dev[s] = amp[s] / h^dim at node
 * (iz[s], ix[s]) and zero elsewhere, for s < nsrc. iz, ix, amp are host
 * arrays (amp NULL = unit amplitude); b_dev is [nsrc][nz][nx].
 * Errors: HZ_ERR_STATE, HZ_ERR_ARG (node outside the grid). */
int  hz_point_rhs(hz_ctx *c, int nsrc, const int *iz, const int *ix,
                  const hz_c128 *amp, hz_c128 *b_dev);

/* A 3D slowness model (Eq. (1) poses the problem in d = 1, 2, 3 dimensions;
 * constant density as in Eq. (2)): nodes (iz, iy, ix) at spacing h, every
 * face of the box absorbing, the same control-volume discretisation as in 1D
 * and 2D (7-point stencil; a node's face weights are the products of the
 * other axes' end weights). m_dev: device, [nz][ny][nx] doubles, copied.
 * Every axis halves on each coarser level. A 3D model is solved by hz_solve
 * with BiCGSTAB or GMRES and the multigrid or no preconditioner (u_dev and
 * b_dev [nfreq][nrhs][nz][ny][nx]); the exact 1D preconditioner returns
 * HZ_ERR_ARG for it. Its misfit, gradient and Gauss-Newton step are the _3d
 * calls below (the 2D calls return HZ_ERR_ARG for a 3D model).
 * Errors: HZ_ERR_ARG (nz, ny or nx < 3, h <= 0, non-finite or non-positive m,
 * more than 2^30 nodes). */
int  hz_set_model_3d(hz_ctx *c, int nz, int ny, int nx, double h, const double *m_dev);

/* Point sources on a 3D model: b_dev[s] = amp[s] / h^3 at node
 * (iz[s], iy[s], ix[s]), zero elsewhere; b_dev is [nsrc][nz][ny][nx].
 * Errors: HZ_ERR_STATE, HZ_ERR_ARG (node outside the grid, model not 3D;
 * hz_point_rhs refuses a 3D model). */
int  hz_point_rhs_3d(hz_ctx *c, int nsrc, const int *iz, const int *iy, const int *ix,
                     const hz_c128 *amp, hz_c128 *b_dev);

/* Solve B(omega_f) u = b for nfreq frequencies (Hz, > 0) times nrhs
 * right-hand sides each, all in one batch. b_dev and u_dev are
 * [nfreq][nrhs][nz][nx] and must not overlap. info (host, optional) receives
 * nfreq*nrhs records. Returns HZ_WARN_NOCONV if some record's status is not
 * HZ_RHS_CONVERGED (its u is the last iterate). nrhs = 0 is an empty batch:
 * nothing is read or written and HZ_OK is returned.
 * Errors: HZ_ERR_ARG, HZ_ERR_SHAPE, HZ_ERR_NOMEM, HZ_ERR_STATE, HZ_ERR_DEVICE. */
int  hz_solve(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
              double alpha, int nrhs, const hz_c128 *b_dev, hz_c128 *u_dev,
              hz_rhs_info *info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hz_solve
 * with the same arguments, results and errors, whose whole solver workspace
 * (Krylov and multigrid vectors, the per-frequency tables and coarse
 * inverses, the slot records and reduction partials) is taken from a static
 * device array of HZ_NOALLOC_BYTES that the library holds on every device it
 * runs on until the process ends. The call itself allocates nothing: no
 * hipMalloc or hipFree, no launch-shape trials (launch shapes the context
 * has already tuned are reused, others take the default shape), no kernel
 * timing and no graphs. The model must have been set by hz_set_model (which
 * allocates the level hierarchy once); the context's own workspace is left
 * as it was. The coarse inverses are formed again on every call.
 * Every call on a device shares that device's array and overwrites it:
 * calls that overlap in time on one device (several contexts, streams or
 * threads) race and must be serialised by the caller.
 * Errors: those of hz_solve, and HZ_ERR_NOMEM (with a message giving the
 * bytes needed) when the workspace exceeds HZ_NOALLOC_BYTES; hz_footprint
 * estimates it. */
#define HZ_NOALLOC_BYTES (64u << 20)
int  hz_solve_noalloc(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
                      double alpha, int nrhs, const hz_c128 *b_dev, hz_c128 *u_dev,
                      hz_rhs_info *info);

/* Misfit of Eq. (4): J = sum over frequencies, shots and receivers of
 * |d_obs - u(receiver)|^2 + lambda * sum m^2, where u solves B u = b for
 * each shot (point source at (src_iz, src_ix) with amplitude src_amp,
 * host arrays, amp NULL = unit). Receivers are nodes (rec_iz, rec_ix), host
 * arrays. d_obs_dev is [nfreq][nsrc][nrec] on the device; d_cal_dev
 * (optional, same shape) receives the modelled data. *J is written on the
 * host. info as in hz_solve (nfreq*nsrc records). */
int  hz_misfit(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
               double alpha, int nsrc, const int *src_iz, const int *src_ix,
               const hz_c128 *src_amp, int nrec, const int *rec_iz, const int *rec_ix,
               const hz_c128 *d_obs_dev, double lambda, double *J,
               hz_c128 *d_cal_dev, hz_rhs_info *info);

/* Misfit and its gradient by the adjoint-state method (Eq. (7) of the
 * paper, the exact derivative of J as written in Eq. (4)):
 *   dJ/dm_i = -2 Re sum_{f,s} delta_i u_i mu_i + 2 lambda m_i,
 *   delta_i = dB_ii/dm_i = j omega g_i/h - 2 omega^2 (1 - j alpha) w_i m_i,
 * with u the forward fields and mu the adjoint fields, B mu = P^T conj(P u -
 * d_obs) (B is complex symmetric: the adjoint solve uses the same solver and
 * preconditioner). Arguments as in hz_misfit; grad_dev is a device [nz][nx]
 * array of doubles (written). info (host, optional) receives 2*nfreq*nsrc
 * records: the forward solves, then the adjoint solves. Frequencies are
 * processed in chunks whose wavefields fit the workspace budget (forward
 * fields are kept only for the chunk being differentiated). */
int  hz_gradient(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
                 double alpha, int nsrc, const int *src_iz, const int *src_ix,
                 const hz_c128 *src_amp, int nrec, const int *rec_iz, const int *rec_ix,
                 const hz_c128 *d_obs_dev, double lambda, double *J, double *grad_dev,
                 hz_rhs_info *info);

/* One Gauss-Newton model update (Eq. (8)-(9)): with the gradient g of J
 * (as in hz_gradient) and the Gauss-Newton operator
 *   H v = 2 Re[G^H G v] + 2 lambda v,   G v = -P B^-1 (delta * u * v),
 * solve H dm = -g by conjugate gradients from dm = 0 (the paper uses CG since
 * the Hessian is dense), at most cg_iters iterations or until the CG residual
 * falls to cg_tol times ||g||. Every CG iteration is one batch of Born solves
 * and one batch of adjoint solves over all shots and frequencies; the forward
 * fields are kept on the device for the whole step. dm_dev (device,
 * [nz][nx] doubles) receives the update (the caller forms m + dm); *J the
 * misfit at m; *cg_done the CG iterations taken; info (optional) the
 * forward-solve records (nfreq*nsrc). Other arguments as in hz_gradient. */
int  hz_gn_step(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
                double alpha, int nsrc, const int *src_iz, const int *src_ix,
                const hz_c128 *src_amp, int nrec, const int *rec_iz, const int *rec_ix,
                const hz_c128 *d_obs_dev, double lambda, int cg_iters, double cg_tol,
                double *J, double *dm_dev, int *cg_done, hz_rhs_info *info);

/* hz_misfit, hz_gradient and hz_gn_step on a 3D model (set by
 * hz_set_model_3d): sources and receivers are nodes (iz, iy, ix), host
 * arrays; the source amplitude is amp / h^3. In delta_i, g_i is the node's
 * exposed boundary face area and w_i its control volume, both in cell units
 * (products of the axes' end weights). grad_dev and dm_dev are device
 * [nz][ny][nx] doubles. Everything else, results and errors as in the 2D
 * calls; each returns HZ_ERR_ARG for a model that is not 3D. */
int  hz_misfit_3d(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
                  double alpha, int nsrc, const int *src_iz, const int *src_iy,
                  const int *src_ix, const hz_c128 *src_amp, int nrec, const int *rec_iz,
                  const int *rec_iy, const int *rec_ix, const hz_c128 *d_obs_dev,
                  double lambda, double *J, hz_c128 *d_cal_dev, hz_rhs_info *info);
int  hz_gradient_3d(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
                    double alpha, int nsrc, const int *src_iz, const int *src_iy,
                    const int *src_ix, const hz_c128 *src_amp, int nrec, const int *rec_iz,
                    const int *rec_iy, const int *rec_ix, const hz_c128 *d_obs_dev,
                    double lambda, double *J, double *grad_dev, hz_rhs_info *info);
int  hz_gn_step_3d(hz_ctx *c, const hz_solve_opts *o, int nfreq, const double *freq_hz,
                   double alpha, int nsrc, const int *src_iz, const int *src_iy,
                   const int *src_ix, const hz_c128 *src_amp, int nrec, const int *rec_iz,
                   const int *rec_iy, const int *rec_ix, const hz_c128 *d_obs_dev,
                   double lambda, int cg_iters, double cg_tol, double *J, double *dm_dev,
                   int *cg_done, hz_rhs_info *info);

/* The level count and damped-Jacobi weights the solver will use for one
 * frequency (host computation, no device work): *levels and w[0..levels-2].
 * w must hold HZ_MAX_LEVELS doubles. The plan: o->levels if set, else halve
 * (n -> ceil(n/2) per axis; with n even the last fine node is interpolated
 * from the last coarse node) until the coarsest level has at most 512
 * unknowns or an axis would drop below 3 nodes; per smoothing level, the
 * largest weight in {0.8,...,0.2} not above o->jacobi_w whose local-Fourier
 * smoothing factor stays <= 1 over the level's kh range.
 * Errors: HZ_ERR_STATE (no model), HZ_ERR_SHAPE (o->levels above what the
 * grid allows: halving while every axis keeps >= 3 nodes; or a coarsest level
 * solved exactly at this frequency with more than HZ_COARSE_MAX unknowns). */
int  hz_plan(const hz_ctx *c, const hz_solve_opts *o, double freq_hz,
             int *levels, double *w);

/* The same plan from the grid and the slowness range alone (host only, no
 * context or device needed): dim, nz, nx, h as in hz_set_model, m_min and
 * m_max the extreme slowness values. Errors: HZ_ERR_ARG, HZ_ERR_SHAPE. */
int  hz_plan_grid(int dim, int nz, int nx, double h, double m_min, double m_max,
                  const hz_solve_opts *o, double freq_hz, int *levels, double *w);

/* ---- single steps of the path, for verification ------------------------ */

/* y = A x on multigrid level `level` (0 = finest) for nrhs vectors, with
 * A = B (op 0, mass shift 1 - j alpha) or A = M (op 1, shift beta1 - j beta2),
 * rediscretised on that level's grid with its injected slowness. */
int  hz_apply(hz_ctx *c, int op, int level, double freq_hz, double alpha,
              double beta1, double beta2, int nrhs, const hz_c128 *x_dev,
              hz_c128 *y_dev);

/* One damped-Jacobi sweep of M on a level: u_out = u_in + w (b - M u_in) / diag(M).
 * u_in_dev may be NULL (u_in = 0). u_out_dev must not alias u_in_dev. */
int  hz_smooth(hz_ctx *c, int level, double freq_hz, double beta1, double beta2,
               double w, int nrhs, const hz_c128 *b_dev, const hz_c128 *u_in_dev,
               hz_c128 *u_out_dev);

/* Weighted-residual restriction: bc = 2^-dim P^T (b - M u) from level to level+1. */
int  hz_restrict(hz_ctx *c, int level, double freq_hz, double beta1, double beta2,
                 int nrhs, const hz_c128 *b_dev, const hz_c128 *u_dev, hz_c128 *bc_dev);

/* Bilinear (1D: linear) prolongation and correction: u += P e, e on level+1. */
int  hz_prolong(hz_ctx *c, int level, int nrhs, const hz_c128 *e_dev, hz_c128 *u_dev);

/* One application of the preconditioner selected by o (V-cycle, exact, or
 * identity) at one frequency: u = V b for nrhs vectors on the finest grid. */
int  hz_precond(hz_ctx *c, const hz_solve_opts *o, double freq_hz, int nrhs,
                const hz_c128 *b_dev, hz_c128 *u_dev);

/* ---- serving ----------------------------------------------------------------
 * A server runs solve requests of any grid size, model and frequencies on one
 * device with continuous batching. Requests the batched BiCGSTAB path takes
 * (2D grids, the multigrid preconditioner, no fixed per-level weights) are
 * grouped by grid and solver options; each group runs in one engine whose
 * slots are lanes of 8 right-hand sides: every (request, frequency) takes
 * ceil(nrhs / 8) lanes and keeps the request's own slowness model. A request
 * that arrives while its group's engine runs joins the running batch between
 * two iterations as soon as enough lanes are free, and leaves it when all its
 * right-hand sides have stopped; the engine stops once idle. Engines of
 * different groups, and requests no engine takes (1D, GMRES, other
 * preconditioners), run on workers of their own, each on its own HIP stream,
 * so their work overlaps on the device. Device memory is admitted against the
 * budget by hz_server_footprint. The result of a request does not depend on
 * the others, bit for bit: every reduction is in a fixed order per right-hand
 * side, and a request joins a batch after an even number of its iterations,
 * so its iterate is advanced in the same order as in hz_solve. */

typedef struct hz_server hz_server;

typedef struct {
    int    device;
    size_t hbm_budget_bytes;  /* device memory the slots may hold together; 0 = no limit */
    int    slots;             /* workers (1..64): engines and single requests running at once */
} hz_server_opts;

typedef struct {
    int           dim, nz, nx;   /* grid, as in hz_set_model */
    double        h;
    const double *m_dev;         /* slowness [nz][nx], device; kept alive by the caller until done */
    int           nfreq;
    const double *freq_hz;       /* host, copied at submission */
    double        alpha;
    int           nrhs;          /* right-hand sides per frequency */
    const hz_c128 *b_dev;        /* [nfreq][nrhs][nz][nx], device, kept alive until done */
    hz_c128      *u_dev;         /* same shape, device, written */
    const hz_solve_opts *opts;   /* host, copied at submission; NULL = defaults */
} hz_request;

/* Device memory a solve of this shape holds (host computation, no device). */
size_t hz_footprint(int dim, int nz, int nx, int nfreq, int nrhs, const hz_solve_opts *o);

/* Device memory the server reserves to run such a request: an engine of its
 * lanes (nfreq * ceil(nrhs / 8)) for a request an engine takes, else its
 * hz_footprint (host computation). A request above the budget is refused. */
size_t hz_server_footprint(int dim, int nz, int nx, int nfreq, int nrhs, const hz_solve_opts *o);

/* Errors: HZ_ERR_ARG (bad device or slot count), HZ_ERR_DEVICE.
 * hbm_budget_bytes = 0: nine tenths of the device memory free at creation. */
int  hz_server_create(hz_server **out, const hz_server_opts *o);
/* Runs the queued requests to completion, then releases every slot. */
void hz_server_destroy(hz_server *s);
/* Queue a request; *ticket identifies it. HZ_ERR_NOMEM if its server
 * footprint exceeds the budget on its own. */
int  hz_server_submit(hz_server *s, const hz_request *rq, long long *ticket);
/* Block until the request is done; info (host, optional) receives
 * nfreq*nrhs records, times (host, optional) three doubles: seconds queued,
 * seconds running, latency (submission to completion). Returns the request's
 * hz_solve status. A ticket can be waited for once: a second wait on it,
 * also one from another thread while the first waits, returns HZ_ERR_ARG. */
int  hz_server_wait(hz_server *s, long long ticket, hz_rhs_info *info, double *times);
/* queued: requests waiting; running: requests on the device (an engine runs
 * many); peak_running: most at once so far; bytes_in_use: device memory the
 * running engines and requests hold. */
int  hz_server_stats(hz_server *s, int *queued, int *running, int *peak_running,
                     size_t *bytes_in_use);

/* ---- measurement --------------------------------------------------------- */

/* kernel classes that can be timed (launches on the finest level) */
#define HZ_KERNEL_SMOOTH   0   /* one damped-Jacobi sweep from a nonzero start (V-cycles whose
                                  smoothing is not fused) */
#define HZ_KERNEL_APPLY    1   /* operator application with fused dot products: B p^ and <r^, v>
                                  (BiCGSTAB), B z (GMRES) */
#define HZ_KERNEL_RESTRICT 2   /* residual and restriction (when not fused into the pre-smoothing) */
#define HZ_KERNEL_PROLONG  3   /* prolongation and correction with the post-sweeps (2D: both) */
#define HZ_KERNEL_UPDATE   4   /* Krylov iterate and residual update (GMRES: the Arnoldi
                                  step's Gram-Schmidt passes and scalars) */
#define HZ_KERNEL_COARSE   5   /* dense coarse solve */
#define HZ_KERNEL_PRESMOOTH 6  /* right-hand side (BiCGSTAB: p = r + beta (p - omega v)) and two
                                  Jacobi sweeps from zero; on 2D grids also the residual and
                                  its restriction */
#define HZ_KERNEL_PRESMOOTH_S 7 /* the same for the BiCGSTAB vector s = r - alpha v */
#define HZ_KERNEL_APPLY_S  8   /* B s^ with <t, s> and <t, t> (BiCGSTAB) */
#define HZ_KERNEL_LEVELS   9   /* every V-cycle launch below the finest level except the dense
                                  coarse solve: smoothing, residual, transfers, and the sweeps
                                  that smooth the coarsest level */

#define HZ_KERNEL_CLASSES  10

/* Start timing the kernel classes whose bit (1 << HZ_KERNEL_*) is set in
 * mask, resetting all totals (mask 0 stops): every later launch of such a
 * class is bracketed by two HIP events on the context's stream.
 * hz_timing_read returns, for one class, the launches and the summed elapsed
 * milliseconds since the start. Errors: HZ_ERR_ARG. */
int  hz_timing_start(hz_ctx *c, unsigned mask);
int  hz_timing_read(hz_ctx *c, int kernel, int *launches, double *total_ms);

/* Text for a return code / the context's last error message. */
const char *hz_status_str(int status);
const char *hz_last_error(const hz_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* HZ_H */
