// The small levels of the 2D V-cycle in two kernels: one workgroup per
// right-hand side walks every level from the first small one down to the
// coarsest (pre-smoothing, residual, restriction; the coarsest level's
// damped-Jacobi sweeps where its frequency smooths it) and, after the dense
// coarse solve, back up (prolongation and correction, post-smoothing), so
// the per-level launches and the gaps between them disappear.
//
// A thread owns the nodes threadIdx.x + k * kSmallBlock of a level and keeps
// their inputs (right-hand side, w / D, slowness) in registers, loaded once
// per level with all loads in flight together; each intermediate vector of
// the level (u1, u2, the residual, u2 + P e, u4) is exchanged through one
// LDS array of the level's size, so a phase reads its neighbours from LDS,
// not from memory.
//
// The arithmetic is that of the per-level kernels: V(2,2) with the two
// pre-sweeps from zero, damped Jacobi in the form (1 - w) u + (w / D)(b +
// (wz sx + wx sz) / h^2) (w / D tabulated per frequency and level), the
// residual with the shifted Laplacian M of the level, full weighting 2^-2 P^T
// of the residual (weight 1 for the last fine node of an even-count axis),
// and bilinear prolongation. With a density (Eq. (1), RHO) the couplings of
// a node come from the level's table (Grid::dc, see RhoC), read where they
// are used (the table is shared by every right-hand side and stays in cache).

#include "hz_device.h"

#include <atomic>

namespace hz {

namespace {

constexpr int kSmallBlock = 1024;
constexpr int kPer = (kSmallNodes + kSmallBlock - 1) / kSmallBlock;  // nodes per thread at most

// weight of a node in its axis (1/2 at an end node)
__device__ __forceinline__ double end_w(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

// one damped-Jacobi update from u at the node and the sums of its existing
// x- and z-neighbours; cz = wz / h^2, cx = wx / h^2, omw = 1 - w
__device__ __forceinline__ double2 jacobi_form(double2 u, double2 b, double2 wd, double2 sx, double2 sz, double cz,
                                               double cx, double omw) {
  const double tx = cz * sx.x + (cx * sz.x + b.x);
  const double ty = cz * sx.y + (cx * sz.y + b.y);
  return c2(omw * u.x + (wd.x * tx - wd.y * ty), omw * u.y + (wd.x * ty + wd.y * tx));
}

// sums of the existing x- and z-neighbours of node p = (iz, ix) in LDS
__device__ __forceinline__ void nbr_sums(const double2* S, int p, int iz, int ix, int nz, int nx, double2& sx,
                                         double2& sz) {
  sx = c2(0.0, 0.0);
  sz = c2(0.0, 0.0);
  if (ix > 0) sx = cadd(sx, S[p - 1]);
  if (ix < nx - 1) sx = cadd(sx, S[p + 1]);
  if (iz > 0) sz = cadd(sz, S[p - nx]);
  if (iz < nz - 1) sz = cadd(sz, S[p + nx]);
}

// the density couplings of node p = (iz, ix) from the level's table
__device__ __forceinline__ RhoC rho_at(const Grid& g, int p, int iz, int ix) {
  const size_t n = (size_t)g.nz * g.nx;
  RhoC c;
  c.l = ix > 0 ? g.dc[p - 1] : 0.0;
  c.r = g.dc[p];
  c.u = iz > 0 ? g.dc[n + p - g.nx] : 0.0;
  c.d = g.dc[n + p];
  return c;
}

// the four neighbours of node p in LDS (zero where missing)
__device__ __forceinline__ void nbrs(const double2* S, int p, int iz, int ix, int nz, int nx, double2& xl, double2& xr,
                                     double2& xu, double2& xd) {
  const double2 z = c2(0.0, 0.0);
  xl = ix > 0 ? S[p - 1] : z;
  xr = ix < nx - 1 ? S[p + 1] : z;
  xu = iz > 0 ? S[p - nx] : z;
  xd = iz < nz - 1 ? S[p + nx] : z;
}

// one damped-Jacobi update at node p of level g from the values in LDS
template <bool RHO>
__device__ __forceinline__ double2 sweep_at(const Grid& g, const double2* S, int p, int iz, int ix, double2 u, double2 b,
                                            double2 wd, double ih2, double omw) {
  if (RHO) {
    double2 xl, xr, xu, xd;
    nbrs(S, p, iz, ix, g.nz, g.nx, xl, xr, xu, xd);
    return jacobi_rho(u, b, wd, rho_at(g, p, iz, ix), xl, xr, xu, xd, ih2, omw);
  }
  double2 sx, sz;
  nbr_sums(S, p, iz, ix, g.nz, g.nx, sx, sz);
  return jacobi_form(u, b, wd, sx, sz, ih2 * end_w(iz, g.nz), ih2 * end_w(ix, g.nx), omw);
}

// bilinear interpolation of coarse e at fine node (iz, ix); the last node of
// an even-count axis takes the last coarse node alone (clamped index)
__device__ __forceinline__ double2 prolong_at(const double2* __restrict__ e, int iz, int ix, int ncx, int ncz) {
  const int Jx = ix >> 1, ox = ix & 1, Jx1 = min(Jx + 1, ncx - 1);
  const int Jz = iz >> 1, oz = iz & 1;
  const double2* r0 = e + Jz * ncx;
  const double2* r1 = (oz && Jz + 1 < ncz) ? r0 + ncx : r0;
  const double2 a0 = r0[Jx], a1 = r0[Jx1], b0 = r1[Jx], b1 = r1[Jx1];
  const double2 a = ox ? cscale(0.5, cadd(a0, a1)) : a0;
  if (!oz) return a;
  const double2 bb = ox ? cscale(0.5, cadd(b0, b1)) : b0;
  return cscale(0.5, cadd(a, bb));
}

}  // namespace

// Descent over levels l0 .. L-2 and the coarsest level's sweeps.
template <bool RHO>
__global__ void __launch_bounds__(kSmallBlock) k_vdown(SmallLevels s, Batch bt) {
  extern __shared__ double2 S[];
  int slot;
  if (!decode_slot_block(bt, slot)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const int t = threadIdx.x;
  for (int l = s.l0; l < s.L - 1; ++l) {
    const Grid g = s.g[l], gc = s.g[l + 1];
    const int n = g.nz * g.nx;
    const double ih2 = 1.0 / (g.h * g.h);
    const double2* b = s.b[l] + (size_t)slot * s.n[l];
    double2* x = s.x[l] + (size_t)slot * s.n[l];
    double2* bc = s.b[l + 1] + (size_t)slot * s.n[l + 1];
    const double2* wdt = f.winv[l];
    const double omw = 1.0 - f.wj[l];
    double2 bk[kPer], wk[kPer], uk[kPer];
    double mk[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = min(t + k * kSmallBlock, n - 1);
      bk[k] = b[p];
      wk[k] = wdt[p];
    }
    // u1 = (w/D) b
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = t + k * kSmallBlock;
      if (p < n) S[p] = cmul(bk[k], wk[k]);
    }
    __syncthreads();
    // u2: the second sweep (the first from zero is u1)
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = t + k * kSmallBlock;
      if (p >= n) continue;
      const int iz = p / g.nx, ix = p - iz * g.nx;
      uk[k] = sweep_at<RHO>(g, S, p, iz, ix, S[p], bk[k], wk[k], ih2, omw);
    }
    __syncthreads();
    // the slowness for the residual (w / D is no longer needed)
#pragma unroll
    for (int k = 0; k < kPer; ++k) mk[k] = model_m(g, f)[min(t + k * kSmallBlock, n - 1)];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = t + k * kSmallBlock;
      if (p >= n) continue;
      S[p] = uk[k];
      x[p] = uk[k];  // the pre-smoothed iterate, for the ascent
    }
    __syncthreads();
    // residual b - M u2
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = t + k * kSmallBlock;
      if (p >= n) continue;
      const int iz = p / g.nx, ix = p - iz * g.nx;
      if (RHO) {
        double2 xl, xr, xu, xd;
        nbrs(S, p, iz, ix, g.nz, g.nx, xl, xr, xu, xd);
        const double om2 = f.omega * f.omega;
        const double gb = g.dc[2 * (size_t)n + p];
        uk[k] = csub(bk[k], apply_m_rho(rho_at(g, p, iz, ix), gb, end_w(iz, g.nz) * end_w(ix, g.nx), mk[k],
                                        -om2 * f.sM_re, -om2 * f.sM_im, f.omega / g.h, ih2, uk[k], xl, xr, xu, xd));
      } else {
        const NodeC c = node_coef<true>(iz, ix, g.nz, g.nx, 1.0 / g.h, mk[k], f.omega, f.sM_re, f.sM_im);
        double2 sx, sz;
        nbr_sums(S, p, iz, ix, g.nz, g.nx, sx, sz);
        uk[k] = csub(bk[k], stencil(c, ih2, uk[k], sx, sz));
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = t + k * kSmallBlock;
      if (p < n) S[p] = uk[k];
    }
    __syncthreads();
    // full weighting to the next level
    const int nc = gc.nz * gc.nx;
    for (int P = t; P < nc; P += kSmallBlock) {
      const int Iz = P / gc.nx, Ix = P - Iz * gc.nx;
      double2 acc = c2(0.0, 0.0);
      for (int dz = -1; dz <= 1; ++dz) {
        const int iz = 2 * Iz + dz;
        if (iz < 0 || iz >= g.nz) continue;
        const double wzt = (dz == 0 || (dz == 1 && 2 * Iz + 2 == g.nz)) ? 1.0 : 0.5;
        double2 row = c2(0.0, 0.0);
        for (int dx = -1; dx <= 1; ++dx) {
          const int ix = 2 * Ix + dx;
          if (ix < 0 || ix >= g.nx) continue;
          const double wxt = (dx == 0 || (dx == 1 && 2 * Ix + 2 == g.nx)) ? 1.0 : 0.5;
          row = cadd(row, cscale(wxt, S[iz * g.nx + ix]));
        }
        acc = cadd(acc, cscale(wzt, row));
      }
      bc[P] = cscale(0.25, acc);
    }
    __syncthreads();
  }
  // coarsest level of a frequency that smooths it: sweeps from zero with the
  // fixed weight s.coarse_w (w / D formed here), ping-ponged between two
  // halves of the LDS array (the coarsest level has at most a quarter of the
  // nodes of level l0, plus its boundary rows and columns), the last one
  // stored to u
  if (!f.coarse_jacobi || s.coarse_sweeps < 1) return;
  const int cl = s.L - 1;
  const Grid g = s.g[cl];
  const int n = g.nz * g.nx;
  const double ih2 = 1.0 / (g.h * g.h);
  const double2* b = s.b[cl] + (size_t)slot * s.n[cl];
  double2* u = s.u[cl] + (size_t)slot * s.n[cl];
  double2* cur = S;
  double2* nxt = S + n;
  for (int sw = 0; sw < s.coarse_sweeps; ++sw) {
    double2* dst = sw + 1 == s.coarse_sweeps ? u : nxt;
    for (int p = t; p < n; p += kSmallBlock) {
      const int iz = p / g.nx, ix = p - iz * g.nx;
      // (node_op reads the density itself: the per-step kernels' arithmetic)
      const NodeOp o = node_op<true>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sM_re, f.sM_im);
      const double2 wdinv = cscale(s.coarse_w, cinv(diag_of<true>(o.c, ih2)));
      if (sw == 0) {
        dst[p] = cmul(b[p], wdinv);
      } else {
        const int nx = g.nx;
        const double2 res = csub(b[p], apply_op_at<true>(g, o, iz, ix, ih2, cur[p], [&](int dz, int dx) {
                                   return cur[p + dz * nx + dx];
                                 }));
        dst[p] = cadd(cur[p], cmul(res, wdinv));
      }
    }
    __syncthreads();
    double2* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

// Ascent over levels L-2 .. l0: u = two sweeps from u2 + P e, with u2 the
// pre-smoothed iterate the descent left in the level's first buffer.
template <bool RHO>
__global__ void __launch_bounds__(kSmallBlock) k_vup(SmallLevels s, Batch bt) {
  extern __shared__ double2 S[];
  int slot;
  if (!decode_slot_block(bt, slot)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const int t = threadIdx.x;
  for (int l = s.L - 2; l >= s.l0; --l) {
    const Grid g = s.g[l], gc = s.g[l + 1];
    const int n = g.nz * g.nx;
    const double ih2 = 1.0 / (g.h * g.h);
    const double2* b = s.b[l] + (size_t)slot * s.n[l];
    const double2* x = s.x[l] + (size_t)slot * s.n[l];
    double2* u = s.u[l] + (size_t)slot * s.n[l];
    const double2* e = s.u[l + 1] + (size_t)slot * s.n[l + 1];
    const double2* wdt = f.winv[l];
    const double omw = 1.0 - f.wj[l];
    double2 bk[kPer], wk[kPer], uk[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = min(t + k * kSmallBlock, n - 1);
      const int iz = p / g.nx, ix = p - iz * g.nx;
      bk[k] = b[p];
      wk[k] = wdt[p];
      uk[k] = cadd(x[p], prolong_at(e, iz, ix, gc.nx, gc.nz));  // u3 = u2 + P e
    }
    // two sweeps from u3; the second is stored to u
    for (int sw = 0; sw < 2; ++sw) {
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int p = t + k * kSmallBlock;
        if (p < n) S[p] = uk[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int p = t + k * kSmallBlock;
        if (p >= n) continue;
        const int iz = p / g.nx, ix = p - iz * g.nx;
        uk[k] = sweep_at<RHO>(g, S, p, iz, ix, uk[k], bk[k], wk[k], ih2, omw);
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int p = t + k * kSmallBlock;
      if (p < n) u[p] = uk[k];
    }
    __syncthreads();  // the next (finer) level reads u as its coarse correction
  }
}

size_t small_levels_lds(const SmallLevels& s) {
  int nmax = 0;
  for (int l = s.l0; l < s.L - 1; ++l) nmax = max(nmax, s.g[l].nz * s.g[l].nx);
  nmax = max(nmax, 2 * s.g[s.L - 1].nz * s.g[s.L - 1].nx);  // the coarsest level's two sweep buffers
  return (size_t)nmax * sizeof(double2);
}

namespace {
// allows the kernel a dynamic LDS size of `bytes` (raised once per process and size)
template <class K>
hipError_t allow_lds(K kernel, size_t bytes, std::atomic<size_t>& allowed) {
  if (bytes <= allowed.load()) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) {
    size_t cur = allowed.load();
    while (cur < bytes && !allowed.compare_exchange_weak(cur, bytes)) {
    }
  }
  return e;
}
std::atomic<size_t> g_allowed[4];  // k_vdown<false, true>, k_vup<false, true>

template <bool RHO>
hipError_t launch_small(bool down, const SmallLevels& s, const Batch& bt, int cap, hipStream_t st) {
  const size_t lds = small_levels_lds(s);
  const auto kernel = down ? k_vdown<RHO> : k_vup<RHO>;
  const hipError_t e = allow_lds(kernel, lds, g_allowed[(down ? 0 : 2) + (RHO ? 1 : 0)]);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, dim3((unsigned)cap), dim3(kSmallBlock), lds, st, s, bt);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_vdown(const SmallLevels& s, const Batch& bt, int cap, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (s.g[s.l0].rho && !s.g[s.l0].dc) return hipErrorInvalidValue;  // a density needs the coupling tables
  return s.g[s.l0].dc ? launch_small<true>(true, s, bt, cap, st) : launch_small<false>(true, s, bt, cap, st);
}

hipError_t launch_vup(const SmallLevels& s, const Batch& bt, int cap, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (s.g[s.l0].rho && !s.g[s.l0].dc) return hipErrorInvalidValue;  // a density needs the coupling tables
  return s.g[s.l0].dc ? launch_small<true>(false, s, bt, cap, st) : launch_small<false>(false, s, bt, cap, st);
}

}  // namespace hz
