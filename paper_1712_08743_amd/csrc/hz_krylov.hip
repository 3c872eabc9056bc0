// HIP kernels of the batched Krylov solvers (gfx950): right-preconditioned
// BiCGSTAB and restarted GMRES(m) over many right-hand sides ("slots") at
// once, the device-side compaction of the active slot list, and the true
// residual. Vector kernels stream complex128 vectors with 16-byte accesses,
// kVecPerThread nodes per thread; per-slot reductions are two-kernel and in
// a fixed order (see store_partial / sum_partials).

#include "hz_device.h"
#include "hz_node3.h"

namespace hz {

__device__ __forceinline__ bool decode_vec(const Batch& bt, int tiles, int& slot, int& tile) {
  return decode_block(bt, tiles, slot, tile);
}

// ---------------------------------------------------------------- BiCGSTAB producers
__global__ void __launch_bounds__(kBlock) k_copy(Batch bt, int tiles, size_t n,
                                                 const double2* __restrict__ x,
                                                 double2* __restrict__ y, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) y[base + i] = x[base + i];
  }
}

// dst = src row by row for nslots slots of an nz x nx grid whose rows have
// pitch sp (slot stride ss) in src and dp (slot stride ds) in dst; dst's
// columns nx .. dp - 1 are set to zero.
__global__ void __launch_bounds__(kBlock) k_repitch(int nz, int nx, const double2* __restrict__ src, int sp,
                                                    size_t ss, double2* __restrict__ dst, int dp, size_t ds,
                                                    size_t total) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const size_t per = (size_t)nz * dp;
  const size_t slot = i / per, rem = i - slot * per;
  const int row = (int)(rem / dp), col = (int)(rem - (size_t)row * dp);
  dst[slot * ds + rem] = col < nx ? src[slot * ss + (size_t)row * sp + col] : c2(0.0, 0.0);
}

// Node i of n in [nz][nx] order at its place in a vector whose rows have
// pitch px (px = 0: the same index). Init and restart walk the nodes in this
// order whatever the pitch, so their sums group as without one.
__device__ __forceinline__ size_t pitched_at(size_t i, int nx, int px) {
  if (px == 0) return i;
  const size_t row = i / (size_t)nx;
  return row * px + (i - row * nx);
}

// x = 0, r = rh = b, p = v = 0 (v null: not stored); partial ||b||^2. b has
// slot stride bstride and rows of nx; the others stride and rows of pitch px
// (0: nx). A pitched vector's padding is not written.
__global__ void __launch_bounds__(kBlock) k_bicg_init(Batch bt, int tiles, size_t n, Reduce rd,
                                                      const double2* __restrict__ b,
                                                      double2* __restrict__ x, double2* __restrict__ r,
                                                      double2* __restrict__ rh, double2* __restrict__ p,
                                                      double2* __restrict__ v, size_t stride, size_t bstride,
                                                      int nx, int px) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride, bbase = (size_t)slot * bstride;
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) {
      const double2 bi = b[bbase + i];
      const size_t a = base + pitched_at(i, nx, px);
      const double2 z = c2(0.0, 0.0);
      x[a] = z;
      r[a] = bi;
      rh[a] = bi;
      p[a] = z;
      if (v) v[a] = z;
      acc[0] += bi.x * bi.x + bi.y * bi.y;
    }
  }
  store_partial<1>(acc, rd, slot, tile);
}

// p_new = r + beta (p_old - omega v)
__global__ void __launch_bounds__(kBlock) k_bicg_p(Batch bt, int tiles, size_t n,
                                                   const double2* __restrict__ r,
                                                   const double2* __restrict__ p_old,
                                                   const double2* __restrict__ v,
                                                   double2* __restrict__ p_new, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const Slot& S = bt.slots[slot];
  const double2 beta = S.beta, om = S.omega;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) {
      const double2 t = csub(p_old[base + i], cmul(om, v[base + i]));
      p_new[base + i] = cadd(r[base + i], cmul(beta, t));
    }
  }
}

// v = B ph; partial <rh, v>.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_bicg_apply_sigma(Grid g, Tiles t, Batch bt, Reduce rd,
                                                             const double2* __restrict__ ph,
                                                             const double2* __restrict__ rh,
                                                             double2* __restrict__ v, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
  const bool dense_rh = bt.slots[slot].rh_nnz < 0;  // else <rh, v> is formed from the sparse list
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    const NodeOp o = node_op<D2>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
    const double2* xs = ph + base;
    const double2 y = apply_op<D2>(g, o, xs, p, iz, ix, 1.0 / (g.h * g.h), xs[p]);
    v[base + p] = y;
    if (dense_rh) {
      const double2 d = cconjmul(rh[base + p], y);
      acc[0] = d.x;
      acc[1] = d.y;
    }
  }
  store_partial<2>(acc, rd, slot, tile);
}

// The per-node coefficients of B at grid node (iz, ix) = p of a 2D grid
// that do not depend on the right-hand side: the slowness and, with a
// density (RHO, Eq. (1)), the couplings and g sqrt(rho) from the level's
// table (Grid::dc). Loaded apart from the stencil so that a kernel can issue
// these loads before its LDS fill and barrier.
struct TileCoef {
  double m;
  RhoC rc;
  double gb;
};
template <bool RHO>
__device__ __forceinline__ TileCoef tile_coef(const Grid& g, const double* m, int iz, int ix, int p) {
  TileCoef c;
  c.m = m[p];
  if (RHO) {
    const size_t n = (size_t)g.nz * g.nx;
    c.rc.l = ix > 0 ? g.dc[p - 1] : 0.0;
    c.rc.r = g.dc[p];
    c.rc.u = iz > 0 ? g.dc[n + p - g.nx] : 0.0;
    c.rc.d = g.dc[n + p];
    c.gb = g.dc[2 * n + p];
  }
  return c;
}

// (B x) at grid node (iz, ix) with coefficients c, x staged in the LDS tile X
// (the node at tile position (lz, lx)). Both kernels that apply B to s^ call
// it, so they form the same values.
template <bool RHO>
__device__ __forceinline__ double2 apply_b_tile(const Grid& g, const FreqTab& f, const double2 (*X)[kHX], int lz,
                                                int lx, int iz, int ix, const TileCoef& c, double ih, double ih2) {
  if (RHO) {
    const double wxz = ((ix == 0 || ix == g.nx - 1) ? 0.5 : 1.0) * ((iz == 0 || iz == g.nz - 1) ? 0.5 : 1.0);
    const double om2 = f.omega * f.omega;
    return apply_m_rho(c.rc, c.gb, wxz, c.m, -om2 * f.sB_re, -om2 * f.sB_im, f.omega * ih, ih2, X[lz + 1][lx + 1],
                       X[lz + 1][lx], X[lz + 1][lx + 2], X[lz][lx + 1], X[lz + 2][lx + 1]);
  }
  const NodeC nc = node_coef<true>(iz, ix, g.nz, g.nx, ih, c.m, f.omega, f.sB_re, f.sB_im);
  double2 sx, sz;
  halo_sums(X, lz, lx, sx, sz);
  return stencil(nc, ih2, X[lz + 1][lx + 1], sx, sz);
}

// LDS-tiled forms (2D): x staged on the tile and its halo, two nodes per thread.
// WHICH 0: v = B ph, partial <rh, v>; WHICH 1: t = B sh, partials <t, s>, <t, t>.
// With y null nothing is stored: WHICH 0 then serves only the slots whose r^
// is dense (the others leave at once) with their partial <rh, B ph>; WHICH 1
// forms only the partials (k_bicg_xr_t forms t again). RHO: with a density
// (Eq. (1)), the couplings from the level's table (Grid::dc).
template <int WHICH, bool RHO>
__global__ void __launch_bounds__(kBlock) k_bicg_apply_t(Grid g, int ntx, int per_slot, Batch bt, Reduce rd,
                                                         const double2* __restrict__ xin,
                                                         const double2* __restrict__ other,
                                                         double2* __restrict__ y, size_t stride) {
  __shared__ double2 X[kHZ][kHX];
  int slot, tile;
  if (!decode_tile(bt, per_slot, slot, tile)) return;
  if (WHICH == 0 && !y && bt.slots[slot].rh_nnz >= 0) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const TileOrg t = tile_org(tile, ntx);
  const size_t base = (size_t)slot * stride;
  // WHICH 0 with a sparse r^: <rh, v> is formed from the list by the reduction kernel
  const bool dots = WHICH == 1 || bt.slots[slot].rh_nnz < 0;
  // the thread's own nodes' inputs are loaded before the halo fill and its
  // barrier, so that their latency overlaps the fill's
  // (node indices: p in the tables, pv in the vectors, whose rows have pitch vp)
  const int vp = vpitch(g);
  double2 ov[kRowsPerThread];
  TileCoef cv[kRowsPerThread];
  const double* m = model_m(g, f);
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int iz = t.z0 + threadIdx.x / kTX + (kBlock / kTX) * r, ix = t.x0 + threadIdx.x % kTX;
    const bool in = iz < g.nz && ix < g.nx;
    const int p = in ? iz * g.nx + ix : 0, pv = in ? iz * vp + ix : 0;
    ov[r] = in && dots ? other[base + pv] : c2(0.0, 0.0);
    cv[r] = tile_coef<RHO>(g, m, in ? iz : 0, in ? ix : 0, p);
  }
  const double2* xs = xin + base;
  fill_halo(X, g, t, [&](int q, int, int) { return xs[q]; });
  __syncthreads();
  const double ih = 1.0 / g.h, ih2 = ih * ih;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int lz = threadIdx.x / kTX + (kBlock / kTX) * r, lx = threadIdx.x % kTX;
    const int iz = t.z0 + lz, ix = t.x0 + lx;
    if (iz >= g.nz || ix >= g.nx) continue;
    const double2 yp = apply_b_tile<RHO>(g, f, X, lz, lx, iz, ix, cv[r], ih, ih2);
    if (y) st_nt(y + base + (size_t)iz * vp + ix, yp);
    if (WHICH == 0) {
      if (dots) {
        const double2 d = cconjmul(ov[r], yp);
        acc[0] += d.x;
        acc[1] += d.y;
      }
    } else {
      const double2 d = cconjmul(yp, ov[r]);
      acc[0] += d.x;
      acc[1] += d.y;
      acc[2] += yp.x * yp.x + yp.y * yp.y;
    }
  }
  store_partial<3>(acc, rd, slot, tile);
}

// 3D grids (hz_node3.h), one node per thread over the row tiling: v = B ph
// with the partial <rh, v> (dense r^ only), t = B sh with <t, s> and <t, t>.
// Every tile stores its partials, zero past the grid.
template <int WHICH>
__global__ void __launch_bounds__(kBlock) k_bicg_apply3(Grid g, Tiles t, Batch bt, Reduce rd,
                                                        const double2* __restrict__ xin,
                                                        const double2* __restrict__ other,
                                                        double2* __restrict__ y, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  const bool dots = WHICH == 1 || bt.slots[slot].rh_nnz < 0;
  double acc[3] = {0.0, 0.0, 0.0};
  int iz, iy, ix;
  size_t p;
  if (node3_of(t, tile, g, iz, iy, ix, p)) {
    const NodeOp3 o = node_op3(iz, iy, ix, g, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
    const double2 yp = apply_op3(g, o, xin + base, p, iz, iy, ix, 1.0 / (g.h * g.h));
    y[base + p] = yp;
    if (WHICH == 0) {
      if (dots) {
        const double2 d = cconjmul(other[base + p], yp);
        acc[0] = d.x;
        acc[1] = d.y;
      }
    } else {
      const double2 d = cconjmul(yp, other[base + p]);
      acc[0] = d.x;
      acc[1] = d.y;
      acc[2] = yp.x * yp.x + yp.y * yp.y;
    }
  }
  store_partial<3>(acc, rd, slot, tile);
}

// s = r - alpha v
__global__ void __launch_bounds__(kBlock) k_bicg_s(Batch bt, int tiles, size_t n,
                                                   const double2* __restrict__ r,
                                                   const double2* __restrict__ v,
                                                   double2* __restrict__ s, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const double2 al = bt.slots[slot].alpha;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) s[base + i] = csub(r[base + i], cmul(al, v[base + i]));
  }
}

// t = B sh; partials <t, s> and <t, t>.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_bicg_apply_omega(Grid g, Tiles t, Batch bt, Reduce rd,
                                                             const double2* __restrict__ sh,
                                                             const double2* __restrict__ s,
                                                             double2* __restrict__ tv, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[3] = {0.0, 0.0, 0.0};
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    const NodeOp o = node_op<D2>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
    const double2* xs = sh + base;
    const double2 y = apply_op<D2>(g, o, xs, p, iz, ix, 1.0 / (g.h * g.h), xs[p]);
    tv[base + p] = y;
    const double2 ts = cconjmul(y, s[base + p]);
    acc[0] = ts.x;
    acc[1] = ts.y;
    acc[2] = y.x * y.x + y.y * y.y;
  }
  store_partial<3>(acc, rd, slot, tile);
}

// r = s - omega t with the partials <rh, r> and ||r||^2, and the iterate.
// XMODE -1: x += alpha ph + omega sh (every iteration). The iterate may also
// be advanced every second iteration (ph and sh of two iterations are kept
// in two buffers each, "rings" 0 and 1): XMODE 0 (ring 0) leaves x alone and
// the reduction kernel records alpha, omega as the slot's pending term;
// XMODE 1 (ring 1) adds the pending term (when there is one) and the
// current one, x += (alpha0 ph0 + omega0 sh0) + (alpha ph + omega sh).
// Streams per node: 4 (s, t / r and, for a dense r^, rh), 9 with x in ring
// 1, 7 every iteration without the rings; on whole tiles the loads of all
// kVecPerThread nodes are issued at once (about 110 VGPRs), so the occupancy
// target is four waves per SIMD.
template <int XMODE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_bicg_xr(Batch bt, int tiles, size_t n, Reduce rd, double2* __restrict__ x, const double2* __restrict__ ph,
          const double2* __restrict__ sh, const double2* __restrict__ ph0, const double2* __restrict__ sh0,
          const double2* __restrict__ s, const double2* __restrict__ t, double2* __restrict__ r,
          const double2* __restrict__ rh, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const Slot& S0 = bt.slots[slot];
  const double2 al = S0.alpha, om = S0.omega;
  const double2 al0 = S0.pend_alpha, om0 = S0.pend_omega;
  const bool pend = XMODE == 1 && S0.pending;
  const bool dense_rh = S0.rh_nnz < 0;  // else <rh, r> is formed from the sparse list
  const size_t base = (size_t)slot * stride;
  double acc[3] = {0.0, 0.0, 0.0};
  const double2 zero = c2(0.0, 0.0);
  auto node = [&](size_t q, double2 xq, double2 phq, double2 shq, double2 ph0q, double2 sh0q, double2 sq,
                  double2 tq, double2 rhq) {
    if (XMODE != 0) {
      double2 dx = cadd(cmul(al, phq), cmul(om, shq));
      if (pend) dx = cadd(cadd(cmul(al0, ph0q), cmul(om0, sh0q)), dx);
      st_nt(x + q, cadd(xq, dx));
    }
    const double2 ri = csub(sq, cmul(om, tq));
    st_nt(r + q, ri);
    const double2 d = cconjmul(rhq, ri);
    acc[0] += d.x;
    acc[1] += d.y;
    acc[2] += ri.x * ri.x + ri.y * ri.y;
  };
  if ((size_t)(tile + 1) * kVecPerThread * kBlock <= n) {
    // whole tile inside the vector: every load of the thread issued before the first use
    double2 X[kVecPerThread], PH[kVecPerThread], SH[kVecPerThread], P0[kVecPerThread], S0v[kVecPerThread],
        S[kVecPerThread], T[kVecPerThread], RH[kVecPerThread];
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e) {
      const size_t q = base + vec_index(tile, e);
      X[e] = XMODE != 0 ? ld_nt(x + q) : zero;
      PH[e] = XMODE != 0 ? ld_nt(ph + q) : zero;
      SH[e] = XMODE != 0 ? ld_nt(sh + q) : zero;
      P0[e] = pend ? ld_nt(ph0 + q) : zero;
      S0v[e] = pend ? ld_nt(sh0 + q) : zero;
      S[e] = ld_nt(s + q);
      T[e] = ld_nt(t + q);
      RH[e] = dense_rh ? ld_nt(rh + q) : zero;
    }
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e)
      node(base + vec_index(tile, e), X[e], PH[e], SH[e], P0[e], S0v[e], S[e], T[e], RH[e]);
  } else {
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e) {
      const size_t i = vec_index(tile, e);
      if (i < n) {
        const size_t q = base + i;
        node(q, XMODE != 0 ? x[q] : zero, XMODE != 0 ? ph[q] : zero, XMODE != 0 ? sh[q] : zero,
             pend ? ph0[q] : zero, pend ? sh0[q] : zero, s[q], t[q], dense_rh ? rh[q] : zero);
      }
    }
  }
  store_partial<3>(acc, rd, slot, tile);
}

// The update of k_bicg_xr on a 2D grid with t = B s^ formed here from an LDS
// copy of s^ and its halo (the stencil of k_bicg_apply_t, which then stores
// no t): r = s - omega t, x as in k_bicg_xr (XMODE), the partials <rh, r>,
// <r, r> per tile of the LDS-staged kernels. s^ at the node comes from the
// tile, so t costs no HBM traffic of its own: per node s^, s / r (and x,
// ph, ph0, sh0 / x in ring 1) instead of s, t / r and s^ again.
template <int XMODE, bool RHO>
__global__ void __launch_bounds__(kBlock) k_bicg_xr_t(Grid g, int ntx, int per_slot, Batch bt, Reduce rd,
                                                      double2* __restrict__ x, const double2* __restrict__ ph,
                                                      const double2* __restrict__ sh,
                                                      const double2* __restrict__ ph0,
                                                      const double2* __restrict__ sh0,
                                                      const double2* __restrict__ s, double2* __restrict__ r,
                                                      const double2* __restrict__ rh, size_t stride) {
  __shared__ double2 X[kHZ][kHX];
  int slot, tile;
  if (!decode_tile(bt, per_slot, slot, tile)) return;
  const Slot& S0 = bt.slots[slot];
  const FreqTab& f = bt.ft[S0.freq];
  const double2 al = S0.alpha, om = S0.omega;
  const double2 al0 = S0.pend_alpha, om0 = S0.pend_omega;
  const bool pend = XMODE == 1 && S0.pending;
  const bool dense_rh = S0.rh_nnz < 0;  // else <rh, r> is formed from the sparse list
  const TileOrg t = tile_org(tile, ntx);
  const size_t base = (size_t)slot * stride;
  // the thread's own nodes' inputs are loaded before the halo fill and its
  // barrier, so that their latency overlaps the fill's
  const double2 zero = c2(0.0, 0.0);
  double2 S[kRowsPerThread], XV[kRowsPerThread], PH[kRowsPerThread], P0[kRowsPerThread], S0v[kRowsPerThread],
      RH[kRowsPerThread];
  TileCoef cv[kRowsPerThread];
  const double* m = model_m(g, f);
  const int vp = vpitch(g);  // row pitch of the vectors (the tables have nx)
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const int iz = t.z0 + threadIdx.x / kTX + (kBlock / kTX) * k, ix = t.x0 + threadIdx.x % kTX;
    const bool in = iz < g.nz && ix < g.nx;
    const int p = in ? iz * g.nx + ix : 0;
    const size_t q = base + (in ? (size_t)iz * vp + ix : 0);
    S[k] = in ? ld_nt(s + q) : zero;
    XV[k] = in && XMODE != 0 ? ld_nt(x + q) : zero;
    PH[k] = in && XMODE != 0 ? ld_nt(ph + q) : zero;
    P0[k] = in && pend ? ld_nt(ph0 + q) : zero;
    S0v[k] = in && pend ? ld_nt(sh0 + q) : zero;
    RH[k] = in && dense_rh ? ld_nt(rh + q) : zero;
    cv[k] = tile_coef<RHO>(g, m, in ? iz : 0, in ? ix : 0, p);
  }
  const double2* shs = sh + base;
  fill_halo(X, g, t, [&](int q, int, int) { return shs[q]; });
  __syncthreads();
  const double ih = 1.0 / g.h, ih2 = ih * ih;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const int lz = threadIdx.x / kTX + (kBlock / kTX) * k, lx = threadIdx.x % kTX;
    const int iz = t.z0 + lz, ix = t.x0 + lx;
    if (iz >= g.nz || ix >= g.nx) continue;
    const size_t q = base + (size_t)iz * vp + ix;
    const double2 tp = apply_b_tile<RHO>(g, f, X, lz, lx, iz, ix, cv[k], ih, ih2);
    const double2 ri = csub(S[k], cmul(om, tp));
    st_nt(r + q, ri);
    if (XMODE != 0) {
      double2 dx = cadd(cmul(al, PH[k]), cmul(om, X[lz + 1][lx + 1]));
      if (pend) dx = cadd(cadd(cmul(al0, P0[k]), cmul(om0, S0v[k])), dx);
      st_nt(x + q, cadd(XV[k], dx));
    }
    const double2 d = cconjmul(RH[k], ri);
    acc[0] += d.x;
    acc[1] += d.y;
    acc[2] += ri.x * ri.x + ri.y * ri.y;
  }
  store_partial<3>(acc, rd, slot, tile);
}

// x += alpha0 ph0 + omega0 sh0 for the slots with a pending term (all slots
// at the end of a solve; the restarting ones before a restart).
__global__ void __launch_bounds__(kBlock) k_bicg_flush(Batch bt, int tiles, size_t n, int only_restart,
                                                       double2* __restrict__ x, const double2* __restrict__ ph0,
                                                       const double2* __restrict__ sh0, size_t stride, int slot0) {
  const int slot = slot0 + (int)(blockIdx.x / tiles);
  const int tile = blockIdx.x - (slot - slot0) * tiles;
  const Slot& S = bt.slots[slot];
  if (!S.pending || (only_restart && S.status != kRestart)) return;
  const double2 al0 = S.pend_alpha, om0 = S.pend_omega;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) {
      const size_t q = base + i;
      x[q] = cadd(x[q], cadd(cmul(al0, ph0[q]), cmul(om0, sh0[q])));
    }
  }
}

// The one restart after a breakdown: rh = r, p = v = 0; partial <r, r>.
// (n nodes in [nz][nx] order; the vectors' rows have pitch px, 0: nx)
__global__ void __launch_bounds__(kBlock) k_bicg_restart(int tiles, size_t n, Batch bt, Reduce rd,
                                                         const double2* __restrict__ r,
                                                         double2* __restrict__ rh,
                                                         double2* __restrict__ p,
                                                         double2* __restrict__ v, size_t stride, int nx, int px) {
  const int slot = blockIdx.x / tiles;
  const int tile = blockIdx.x - slot * tiles;
  if (bt.slots[slot].status != kRestart) return;
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) {
      const size_t a = base + pitched_at(i, nx, px);
      const double2 ri = r[a];
      rh[a] = ri;
      p[a] = c2(0.0, 0.0);
      if (v) v[a] = c2(0.0, 0.0);
      const double2 d = cconjmul(ri, ri);
      acc[0] += d.x;
      acc[1] += d.y;
    }
  }
  store_partial<2>(acc, rd, slot, tile);
}

// The sparse list of r^ = b (one block per slot): the nonzeros are found in
// one coalesced pass and appended to an LDS list in any order, then each is
// written at its rank by node index, so the list is in ascending order
// whatever order the appends took. More than kShadowMax nonzeros:
// rh_nnz = -1 (r^ stays a dense vector).
__global__ void __launch_bounds__(kBlock) k_rh_sparse(size_t n, Batch bt, const double2* __restrict__ b,
                                                      int* __restrict__ idx, double2* __restrict__ val,
                                                      size_t stride, int slot0) {
  __shared__ int count;
  __shared__ int sidx[kShadowMax];
  __shared__ double2 sval[kShadowMax];
  const int slot = slot0 + (int)blockIdx.x;
  const double2* bs = b + (size_t)slot * stride;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (size_t i = threadIdx.x; i < n; i += kBlock) {
    const double2 bi = bs[i];
    if (bi.x != 0.0 || bi.y != 0.0) {
      const int k = atomicAdd(&count, 1);
      if (k < kShadowMax) {
        sidx[k] = (int)i;
        sval[k] = bi;
      }
    }
  }
  __syncthreads();
  const int total = count;
  if (threadIdx.x == 0) bt.slots[slot].rh_nnz = total <= kShadowMax ? total : -1;
  if (total > kShadowMax) return;
  for (int k = threadIdx.x; k < total; k += kBlock) {
    const int ik = sidx[k];
    int rank = 0;
    for (int j = 0; j < total; ++j) rank += sidx[j] < ik;
    idx[(size_t)slot * kShadowMax + rank] = ik;
    val[(size_t)slot * kShadowMax + rank] = sval[k];
  }
}

// ---------------------------------------------------------------- BiCGSTAB scalars
// One block per slot: fixed-order sum of the producer's partials, then the
// scalar step of the method (van der Vorst's BiCGSTAB, right-preconditioned):
//   init:    bnorm2, rho = ||b||^2, beta = 0 (alpha = omega = 1; the first p is r)
//   sigma:   alpha = rho / <rh, v> (sigma-B: v = B ph)
//   omega:   omega = <t, s> / <t, t>
//   step:    ||r|| test, breakdown / maxit checks, rho' = <rh, r>,
//            beta = (rho'/rho)(alpha/omega)
//   restart: rho = <r, r>, beta = 0; rh = r done by the producer
__global__ void __launch_bounds__(kBlock) k_bicg_fin(int which, int tiles, Batch bt, Reduce rd,
                                                     double tol, int maxit, const double2* __restrict__ vec,
                                                     size_t stride, int ring, int restart_at, Grid g) {
  int slot;
  if (which == kFinRestart) {
    slot = blockIdx.x;
    if (bt.slots[slot].status != kRestart) return;
  } else if (!decode_slot_block(bt, slot)) {
    return;
  }
  // <rh, v> (sigma) or <rh, r> (step) from r^'s sparse list, in list order,
  // in place of the producer's partials (which hold zeros there). Sigma
  // with vec = ph (kFinSigmaB) forms v = B ph at the list's nodes, and its
  // partials are read only where r^ is dense (no producer wrote them
  // otherwise).
  const int nnz = bt.slots[slot].rh_nnz;
  const bool form_b = which == kFinSigmaB;
  const bool sparse = (which == kFinSigma || form_b || which == kFinStep) && nnz >= 0;
  const bool use_partials = !(form_b && sparse);
  double acc[3] = {0.0, 0.0, 0.0};
  const double* src = rd.partials + (size_t)slot * rd.max_tiles * kPartialWidth;
  for (int k = threadIdx.x; k < tiles && use_partials; k += blockDim.x) {
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] += src[(size_t)k * kPartialWidth + q];
  }
  if (sparse) {
    const int* idx = bt.rh_idx + (size_t)slot * kShadowMax;
    const double2* val = bt.rh_val + (size_t)slot * kShadowMax;
    const double2* vs = vec + (size_t)slot * stride;
    const FreqTab& f = bt.ft[bt.slots[slot].freq];
    // the list holds node indices iz * nx + ix (of the tables); with a grid
    // (form_b, and every 2D step reduction) the vector's rows have pitch vp
    const int vp = g.nx > 0 ? vpitch(g) : 0;
    for (int k = threadIdx.x; k < nnz; k += blockDim.x) {
      const int p = idx[k];
      const int iz = g.nx > 0 ? p / g.nx : 0, ix = p - iz * g.nx;
      const int pv = g.nx > 0 ? iz * vp + ix : p;
      double2 y;
      if (form_b) {
        const NodeOp o = node_op<true>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
        y = apply_op_at<true>(g, o, iz, ix, 1.0 / (g.h * g.h), vs[pv],
                              [&](int dz, int dx) { return vs[pv + dz * vp + dx]; });
      } else {
        y = vs[pv];
      }
      const double2 d = cconjmul(val[k], y);
      acc[0] += d.x;
      acc[1] += d.y;
    }
  }
  block_sum<3>(acc);
  if (threadIdx.x != 0) return;
  Slot& S = bt.slots[slot];
  switch (which) {
    case kFinInit: {
      const double b2 = acc[0];
      S.t0 = wall_clock64();
      S.t1 = S.t0;
      S.bnorm2 = b2;
      S.rnorm2 = b2;
      S.iters = 0;
      S.restarted = 0;
      S.alpha = c2(1.0, 0.0);
      S.omega = c2(1.0, 0.0);
      if (!isfinite(b2)) {
        S.status = kNonfinite;
      } else if (b2 == 0.0) {
        S.status = kConverged;
      } else {
        S.rho = c2(b2, 0.0);
        S.beta = c2(0.0, 0.0);  // the first p is r
      }
      break;
    }
    case kFinSigma:
    case kFinSigmaB: {
      const double2 sigma = c2(acc[0], acc[1]);
      if (!cfinite(sigma)) {
        S.status = kNonfinite;
      } else if (czero(sigma)) {
        S.status = S.restarted ? kBreakdown : kRestart;
      } else {
        S.alpha = cdiv(S.rho, sigma);
      }
      break;
    }
    case kFinOmega: {
      const double tt = acc[2];
      const double2 om = tt != 0.0 ? c2(acc[0] / tt, acc[1] / tt) : c2(0.0, 0.0);
      if (!cfinite(S.alpha) || !cfinite(om)) {
        S.status = kNonfinite;
      } else {
        S.omega = om;
      }
      break;
    }
    case kFinStep: {
      // the update just done in ring 0 left alpha ph + omega sh pending; ring 1 added it
      if (ring == 0) {
        S.pend_alpha = S.alpha;
        S.pend_omega = S.omega;
        S.pending = 1;
      } else if (ring == 1) {
        S.pending = 0;
      }
      S.iters += 1;
      S.t1 = wall_clock64();
      S.rnorm2 = acc[2];
      const double rn = sqrt(acc[2]);
      const double2 rho_new = c2(acc[0], acc[1]);
      if (!isfinite(rn)) {
        S.status = kNonfinite;
      } else if (rn <= tol * sqrt(S.bnorm2)) {
        S.status = kConverged;
      } else if (czero(S.omega)) {
        S.status = S.restarted ? kBreakdown : (S.iters >= maxit ? kMaxit : kRestart);
      } else if (S.iters >= maxit) {
        S.status = kMaxit;
      } else if (!cfinite(rho_new)) {
        S.status = kNonfinite;
      } else if (czero(rho_new) || (restart_at > 0 && S.iters == restart_at && !S.restarted)) {
        S.status = S.restarted ? kBreakdown : kRestart;
      } else {
        S.beta = cmul(cdiv(rho_new, S.rho), cdiv(S.alpha, S.omega));
        S.rho = rho_new;
      }
      break;
    }
    case kFinRestart: {
      const double2 rho = c2(acc[0], acc[1]);
      S.restarted = 1;
      S.rh_nnz = -1;  // r^ = r from here on, dense
      S.pending = 0;  // added to x by the flush before the restart
      S.alpha = c2(1.0, 0.0);
      S.omega = c2(1.0, 0.0);
      if (!cfinite(rho)) {
        S.status = kNonfinite;
      } else if (czero(rho)) {
        S.status = kBreakdown;
      } else {
        S.rho = rho;
        S.beta = c2(0.0, 0.0);  // the first p after the restart is r
        S.status = kActive;
      }
      break;
    }
    default:
      break;
  }
}

// Rebuild the active list (ascending slot ids of active slots in want_phase)
// and the host summary.
__global__ void __launch_bounds__(1024) k_compact(int nslots, int nrhs, int nfreq,
                                                  const Slot* __restrict__ slots,
                                                  int* __restrict__ active, int* __restrict__ nactive,
                                                  int* __restrict__ fstart, Summary* sum, int want_phase) {
  __shared__ int wsum[16];
  __shared__ int wres[16];
  __shared__ int woth[16];
  __shared__ int wden[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  int nres_local = 0, noth_local = 0, nden_local = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int b0 = 0; b0 < nslots; b0 += blockDim.x) {
    const int i = b0 + threadIdx.x;
    const int st = i < nslots ? slots[i].status : kConverged;
    const int ph = i < nslots ? slots[i].phase : 0;
    const int a = (st == kActive) && (ph == want_phase);
    nres_local += (st == kRestart);
    noth_local += (st == kActive) && (ph != want_phase);
    nden_local += a && slots[i].rh_nnz < 0;
    int x = a;  // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int before = carry;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    if (a) active[before + x - 1] = i;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wsum[w];
      carry += tot;
    }
    __syncthreads();
  }
  for (int off = 32; off > 0; off >>= 1) {
    nres_local += __shfl_xor(nres_local, off, 64);
    noth_local += __shfl_xor(noth_local, off, 64);
    nden_local += __shfl_xor(nden_local, off, 64);
  }
  if (lane == 0) {
    wres[wid] = nres_local;
    woth[wid] = noth_local;
    wden[wid] = nden_local;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nr = 0, no = 0, nd = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      nr += wres[w];
      no += woth[w];
      nd += wden[w];
    }
    *nactive = carry;
    sum->nactive = carry;
    sum->nrestart = nr;
    sum->nother = no;
    sum->ndense = nd;
  }
  // per-frequency ranges of the (ascending, frequency-major) list
  const int total = carry;
  for (int f = threadIdx.x; f <= nfreq; f += blockDim.x) {
    const int key = f * nrhs;
    int lo = 0, hi = total;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (active[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    fstart[f] = lo;
  }
}

// ---------------------------------------------------------------- true residual
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_true_residual(Grid g, Tiles t, Batch bt, Reduce rd,
                                                          const double2* __restrict__ b,
                                                          const double2* __restrict__ x, size_t stride) {
  // every slot of the list, whatever its status (XCD-aware tile order)
  const int xcd = blockIdx.x % kXcd, k = blockIdx.x / kXcd;
  const int chunk = xcd_chunk(t.per_slot);
  const int si = k / chunk;
  const int tile = xcd * chunk + (k - si * chunk);
  if (tile >= t.per_slot || si >= *bt.nactive) return;
  const int slot = bt.active[si];
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    const NodeOp o = node_op<D2>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
    const double2* xs = x + base;
    const double2 y = apply_op<D2>(g, o, xs, p, iz, ix, 1.0 / (g.h * g.h), xs[p]);
    const double2 bp = b[base + p];
    const double2 rr = csub(bp, y);
    acc[0] = rr.x * rr.x + rr.y * rr.y;
    acc[1] = bp.x * bp.x + bp.y * bp.y;
  }
  store_partial<2>(acc, rd, slot, tile);
}

// ||b - B x||^2 and ||b||^2 on a 3D grid (as k_true_residual)
__global__ void __launch_bounds__(kBlock) k_true_residual3(Grid g, Tiles t, Batch bt, Reduce rd,
                                                           const double2* __restrict__ b,
                                                           const double2* __restrict__ x, size_t stride) {
  const int xcd = blockIdx.x % kXcd, k = blockIdx.x / kXcd;
  const int chunk = xcd_chunk(t.per_slot);
  const int si = k / chunk;
  const int tile = xcd * chunk + (k - si * chunk);
  if (tile >= t.per_slot || si >= *bt.nactive) return;
  const int slot = bt.active[si];
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
  int iz, iy, ix;
  size_t p;
  if (node3_of(t, tile, g, iz, iy, ix, p)) {
    const NodeOp3 o = node_op3(iz, iy, ix, g, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
    const double2 y = apply_op3(g, o, x + base, p, iz, iy, ix, 1.0 / (g.h * g.h));
    const double2 bp = b[base + p];
    const double2 rr = csub(bp, y);
    acc[0] = rr.x * rr.x + rr.y * rr.y;
    acc[1] = bp.x * bp.x + bp.y * bp.y;
  }
  store_partial<2>(acc, rd, slot, tile);
}

__global__ void __launch_bounds__(kBlock) k_true_residual_fin(int tiles, Batch bt, Reduce rd,
                                                              double* __restrict__ out) {
  const int si = blockIdx.x;
  if (si >= *bt.nactive) return;
  const int slot = bt.active[si];
  double acc[2];
  sum_partials<2>(acc, rd, slot, tiles);
  if (threadIdx.x == 0) {
    out[2 * slot] = acc[0];
    out[2 * slot + 1] = acc[1];
  }
}

// ---------------------------------------------------------------- GMRES(m)
// Right-preconditioned restarted GMRES, one Arnoldi process per slot, all
// slots of a cycle in lockstep. The basis vector i of slot s lives at
// V + i * vstride + s * stride. Orthogonalisation is classical Gram-Schmidt
// applied twice with the second pass of each vector delayed to the next
// step (the DCGS2 scheme of Swirydowicz, Langou, Ananthan, Yang and Thomas,
// low-synchronisation Gram-Schmidt for GMRES): step j holds u_j, the first
// pass's result for the last product, and applies the operator to u_j
// itself. One pass over the basis gives s = V^H u_j, ||u_j||^2, p = V^H z
// and <u_j, z> for z = B M^-1 u_j; from these scalars alone come u_j's second
// pass (v_j = (u_j - V s) / r, r^2 = ||u_j||^2 - ||s||^2, completing column
// j - 1 of the Hessenberg matrix: its Givens rotation and the convergence
// test are made then) and the first pass of the next product (B M^-1 v_j =
// (z - V H s) / r by the Arnoldi relation of the finished columns). A second
// pass writes v_j and u_{j+1}. Every per-slot sum is a fixed-order
// two-kernel reduction.

// r = b - B x (x = 0 on the first cycle, which also zeroes x) into V_0;
// partial ||r||^2.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_gm_residual(Grid g, Tiles t, Batch bt, Reduce rd,
                                                        int first, const double2* __restrict__ b,
                                                        double2* __restrict__ x,
                                                        double2* __restrict__ v0, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const size_t base = (size_t)slot * stride;
  double acc[1] = {0.0};
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    double2 r;
    if (first) {
      x[base + p] = c2(0.0, 0.0);
      r = b[base + p];
    } else {
      const FreqTab& f = bt.ft[bt.slots[slot].freq];
      const NodeOp o = node_op<D2>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
      const double2* xs = x + base;
      r = csub(b[base + p], apply_op<D2>(g, o, xs, p, iz, ix, 1.0 / (g.h * g.h), xs[p]));
    }
    v0[base + p] = r;
    acc[0] = r.x * r.x + r.y * r.y;
  }
  store_partial<1>(acc, rd, slot, tile);
}

// The same on a 3D grid (row tiling, hz_node3.h).
__global__ void __launch_bounds__(kBlock) k_gm_residual3(Grid g, Tiles t, Batch bt, Reduce rd, int first,
                                                         const double2* __restrict__ b, double2* __restrict__ x,
                                                         double2* __restrict__ v0, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
  double acc[1] = {0.0};
  int iz, iy, ix;
  size_t p;
  if (node3_of(t, tile, g, iz, iy, ix, p)) {
    double2 r;
    if (first) {
      x[base + p] = c2(0.0, 0.0);
      r = b[base + p];
    } else {
      const FreqTab& f = bt.ft[bt.slots[slot].freq];
      const NodeOp3 o = node_op3(iz, iy, ix, g, p, model_m(g, f)[p], f.omega, f.sB_re, f.sB_im);
      r = csub(b[base + p], apply_op3(g, o, x + base, p, iz, iy, ix, 1.0 / (g.h * g.h)));
    }
    v0[base + p] = r;
    acc[0] = r.x * r.x + r.y * r.y;
  }
  store_partial<1>(acc, rd, slot, tile);
}

// Cycle start: beta = ||r||, g = (beta, 0, ...), or a final status.
__global__ void __launch_bounds__(kBlock) k_gm_residual_fin(int tiles, Batch bt, Reduce rd, Gmres gm,
                                                            int first, double tol, int maxit) {
  int slot;
  if (!decode_slot_block(bt, slot)) return;
  double acc[1];
  sum_partials<1>(acc, rd, slot, tiles);
  if (threadIdx.x != 0) return;
  Slot& S = bt.slots[slot];
  if (first) {
    S.bnorm2 = acc[0];
    S.t0 = wall_clock64();
    S.t1 = S.t0;
    S.iters = 0;
    S.restarted = 0;
  }
  S.rnorm2 = acc[0];
  const double beta = sqrt(acc[0]);
  if (!isfinite(beta)) {
    S.status = kNonfinite;
  } else if (S.bnorm2 == 0.0 || beta <= tol * sqrt(S.bnorm2)) {
    S.status = kConverged;
  } else if (S.iters >= maxit) {
    S.status = kMaxit;
  } else {
    S.phase = 0;
    S.cyc_k = 0;
    S.scal = c2(beta, 0.0);
    double2* gg = gm.g + (size_t)slot * (gm.m + 1);
    gg[0] = c2(beta, 0.0);
    for (int i = 1; i <= gm.m; ++i) gg[i] = c2(0.0, 0.0);
  }
}

// v *= 1 / scal (the newest basis vector's norm); a zero norm leaves v alone.
__global__ void __launch_bounds__(kBlock) k_gm_scale(Batch bt, int tiles, size_t n, double2* __restrict__ v,
                                                     size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const double d = bt.slots[slot].scal.x;
  if (d == 0.0) return;
  const double inv = 1.0 / d;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) v[base + i] = cscale(inv, v[base + i]);
  }
}

// Sum K doubles over the 64 lanes of a wave in a fixed order; valid in every lane.
template <int K>
__device__ __forceinline__ void wave_sum(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  }
}

// The step's one pass over the basis (partials per tile of kGmDotNodes
// nodes, width gm.width): s_i = <V_i, u> at 2i, p_i = <V_i, z> at 2 (j + i)
// (i < j), ||u||^2 at 4j and <u, z> at 4j + 1 for u = V_j (the first pass's
// result) and z = B M^-1 u; z null (the finishing pass of a cycle): s and
// ||u||^2 only. The basis is taken kGmChunk vectors at a time; the thread's
// nodes of u and z stay in registers. Each wave reduces its own sums and
// keeps them in LDS (4j + 3 doubles per wave), so the waves of a block meet
// only once, at the end, where the tile's partials are the sums over the
// waves in wave order.
constexpr int kGmE = 4;      // nodes per thread of the dot pass
constexpr int kGmChunk = 1;  // basis vectors per pass over a tile
constexpr int kGmDotNodes = kGmE * kBlock;
constexpr int kWaves = kBlock / 64;

// six waves per SIMD (74 VGPRs): the fastest of the 2 to 8 measured
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_gm_dots2(Batch bt, int tiles, size_t n, Gmres gm, int j, const double2* __restrict__ V, size_t vstride,
           const double2* __restrict__ z, size_t stride) {
  extern __shared__ double wsum[];  // [kWaves][4j + 3]
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const int nsum = 4 * j + 3;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double* mine = wsum + wid * nsum;
  const size_t base = (size_t)slot * stride;
  const double2* u = V + (size_t)j * vstride + base;
  const double2* zs = z ? z + base : nullptr;
  const size_t i0 = (size_t)tile * kGmDotNodes + threadIdx.x;
  double2 ur[kGmE], zr[kGmE];  // the thread's nodes of u and z, held across the chunks
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const size_t i = i0 + (size_t)e * kBlock;
    ur[e] = i < n ? u[i] : c2(0.0, 0.0);
    zr[e] = i < n && zs ? zs[i] : c2(0.0, 0.0);
  }
  for (int c0 = 0; c0 < j; c0 += kGmChunk) {
    double acc[4 * kGmChunk];
#pragma unroll
    for (int q = 0; q < 4 * kGmChunk; ++q) acc[q] = 0.0;
#pragma unroll
    for (int e = 0; e < kGmE; ++e) {
      const size_t i = i0 + (size_t)e * kBlock;
      if (i < n) {
        const double2 ui = ur[e];
        const double2 zi = zr[e];
#pragma unroll
        for (int q = 0; q < kGmChunk; ++q) {
          if (c0 + q < j) {
            const double2 vq = V[(size_t)(c0 + q) * vstride + base + i];
            const double2 ds = cconjmul(vq, ui), dp = cconjmul(vq, zi);
            acc[4 * q] += ds.x;
            acc[4 * q + 1] += ds.y;
            acc[4 * q + 2] += dp.x;
            acc[4 * q + 3] += dp.y;
          }
        }
      }
    }
    wave_sum<4 * kGmChunk>(acc);
    if (lane == 0) {
      for (int q = 0; q < kGmChunk && c0 + q < j; ++q) {
        mine[2 * (c0 + q)] = acc[4 * q];
        mine[2 * (c0 + q) + 1] = acc[4 * q + 1];
        mine[2 * (j + c0 + q)] = acc[4 * q + 2];
        mine[2 * (j + c0 + q) + 1] = acc[4 * q + 3];
      }
    }
  }
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < kGmE; ++e) {
    const double2 ui = ur[e];
    acc[0] += ui.x * ui.x + ui.y * ui.y;
    const double2 d = cconjmul(ui, zr[e]);
    acc[1] += d.x;
    acc[2] += d.y;
  }
  wave_sum<3>(acc);
  if (lane == 0) {
    mine[4 * j] = acc[0];
    mine[4 * j + 1] = acc[1];
    mine[4 * j + 2] = acc[2];
  }
  __syncthreads();
  double* part = gm.partials + ((size_t)slot * gm.max_tiles + tile) * gm.width;
  for (int v = threadIdx.x; v < nsum; v += kBlock) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) a += wsum[w * nsum + v];
    part[v] = a;
  }
}

__device__ __forceinline__ void givens(double2 a, double2 b, double& c, double2& s) {
  const double na = sqrt(a.x * a.x + a.y * a.y), nb = sqrt(b.x * b.x + b.y * b.y);
  if (nb == 0.0) {
    c = 1.0;
    s = c2(0.0, 0.0);
  } else if (na == 0.0) {
    c = 0.0;
    s = c2(1.0, 0.0);
  } else {
    const double nu = hypot(na, nb);
    c = na / nu;
    // s = (a / |a|) conj(b) / nu
    const double2 ua = c2(a.x / na, a.y / na);
    s = cscale(1.0 / nu, cmul(ua, c2(b.x, -b.y)));
  }
}

// The step's scalars, per slot (one block): the partials summed in tile
// order, then (thread 0) for j >= 1 u_j's second pass r = sqrt(||u_j||^2 -
// ||s||^2) completing column j - 1 of the Arnoldi matrix Hu (Hu[i, j-1] += s_i,
// Hu[j, j-1] = r), its rotated copy in H with the Givens rotations and g, the
// iteration count and the convergence test (or, with finish, the cycle's
// end); where the slot goes on, the first pass of column j from the scalars
// (thread k its row): h_k = (p_k - (Hu s)_k) / r (k < j) and h_j = ((<u_j, z> -
// s^H p) / r - (Hu s)_j) / r, and the update coefficients c = Hu s / r + h
// (hc[1]) beside s (hc[0]) and scal = r for k_gm_update2. j = 0: V_0 is final,
// h_0 = <V_0, z>. Shared memory: 4j + 3 doubles of sums, then column j - 1
// (j + 1 complex) and two flags.
__global__ void __launch_bounds__(kBlock) k_gm_fin2(int tiles, Batch bt, Gmres gm, int j, double tol, int maxit,
                                                    int finish) {
  extern __shared__ double sum[];
  int slot;
  if (!decode_slot_block(bt, slot)) return;
  const double* src = gm.partials + (size_t)slot * gm.max_tiles * gm.width;
  const int nsum = 4 * j + 3;
  for (int v = threadIdx.x; v < nsum; v += blockDim.x) {
    // tile order; eight loads in flight at a time
    double a = 0.0;
    int tt = 0;
    for (; tt + 8 <= tiles; tt += 8) {
      double x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = src[(size_t)(tt + k) * gm.width + v];
#pragma unroll
      for (int k = 0; k < 8; ++k) a += x[k];
    }
    for (; tt < tiles; ++tt) a += src[(size_t)tt * gm.width + v];
    sum[v] = a;
  }
  double2* colj = reinterpret_cast<double2*>(sum + ((nsum + 1) & ~1));  // column j - 1 of Hu
  double* flag = reinterpret_cast<double*>(colj + j + 1);               // [0]: go on, [1]: r
  __syncthreads();
  Slot& S = bt.slots[slot];
  const int m1 = gm.m + 1;
  double2* Hu = gm.Hu + (size_t)slot * m1 * gm.m;  // column i at Hu + i * m1
  double2* H = gm.H + (size_t)slot * m1 * gm.m;
  double2* sv = gm.hc + (size_t)slot * 2 * m1;
  double2* cv = sv + m1;
  const double2 q = c2(sum[4 * j + 1], sum[4 * j + 2]);
  auto s_at = [&](int i) { return c2(sum[2 * i], sum[2 * i + 1]); };
  auto p_at = [&](int i) { return c2(sum[2 * (j + i)], sum[2 * (j + i) + 1]); };
  if (j == 0) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < m1; ++k) Hu[k] = c2(0.0, 0.0);
    Hu[0] = q;
    cv[0] = q;
    S.scal = c2(1.0, 0.0);
    return;
  }
  if (threadIdx.x == 0) {
    flag[0] = 0.0;
    double nrm2 = sum[4 * j];
    for (int i = 0; i < j; ++i) {
      const double2 si = s_at(i);
      nrm2 -= si.x * si.x + si.y * si.y;
    }
    const double r = sqrt(fmax(nrm2, 0.0));
    flag[1] = r;
    // column j - 1 completed, then rotated
    double2* Huc = Hu + (size_t)(j - 1) * m1;
    for (int i = 0; i < j; ++i) {
      colj[i] = cadd(Huc[i], s_at(i));
      Huc[i] = colj[i];
    }
    colj[j] = c2(r, 0.0);
    Huc[j] = colj[j];
    double2* Hc = H + (size_t)(j - 1) * m1;
    for (int i = 0; i <= j; ++i) Hc[i] = colj[i];
    double* cs = gm.cs + (size_t)slot * gm.m;
    double2* sn = gm.sn + (size_t)slot * gm.m;
    double2* gg = gm.g + (size_t)slot * m1;
    const int k = j - 1;
    for (int i = 0; i < k; ++i) {
      const double2 a = Hc[i], bb = Hc[i + 1];
      Hc[i] = cadd(cscale(cs[i], a), cmul(sn[i], bb));
      Hc[i + 1] = csub(cscale(cs[i], bb), cmul(c2(sn[i].x, -sn[i].y), a));
    }
    double ck;
    double2 sk;
    givens(Hc[k], Hc[k + 1], ck, sk);
    cs[k] = ck;
    sn[k] = sk;
    Hc[k] = cadd(cscale(ck, Hc[k]), cmul(sk, Hc[k + 1]));
    Hc[k + 1] = c2(0.0, 0.0);
    const double2 gk = gg[k];
    gg[k + 1] = cmul(c2(-sk.x, sk.y), gk);  // -conj(s) g_k
    gg[k] = cscale(ck, gk);
    S.iters += 1;
    S.cyc_k = j;
    S.t1 = wall_clock64();
    const double est = sqrt(gg[k + 1].x * gg[k + 1].x + gg[k + 1].y * gg[k + 1].y);
    if (!isfinite(est) || !isfinite(r)) {
      S.status = kNonfinite;
    } else if (finish || r == 0.0 || est <= tol * sqrt(S.bnorm2) || S.iters >= maxit) {
      S.phase = 1;
    } else {
      flag[0] = 1.0;
      S.scal = c2(r, 0.0);
    }
  }
  __syncthreads();
  if (flag[0] == 0.0) return;
  // first pass of column j: h = V^H (B M^-1 v_j) from the scalars, with
  // B M^-1 v_j = (z - sum_{i<j} s_i B M^-1 V_i) / r = (z - V (Hu s)) / r
  const double ir = 1.0 / flag[1];
  double2* Hn = Hu + (size_t)j * m1;
  for (int kk = threadIdx.x; kk < m1; kk += blockDim.x) {
    if (kk > j) {
      Hn[kk] = c2(0.0, 0.0);
      continue;
    }
    double2 hs = c2(0.0, 0.0);  // (Hu s)_kk over the finished columns i >= kk - 1
    for (int i = max(kk - 1, 0); i < j; ++i)
      hs = cadd(hs, cmul(i == j - 1 ? colj[kk] : Hu[(size_t)i * m1 + kk], s_at(i)));
    double2 num;
    if (kk < j) {
      num = p_at(kk);
    } else {
      double2 vz = q;  // <v_j, z> r
      for (int i = 0; i < j; ++i) vz = csub(vz, cconjmul(s_at(i), p_at(i)));
      num = cscale(ir, vz);
    }
    const double2 h = cscale(ir, csub(num, hs));
    Hn[kk] = h;
    cv[kk] = cadd(cscale(ir, hs), h);
    if (kk < j) sv[kk] = s_at(kk);
  }
}

// The step's second pass over the basis, for the slots that go on: v_j =
// (u_j - sum_{i<j} s_i V_i) / r into V_j, and the next first-pass result
// u_{j+1} = z / r - sum_{i<j} c_i V_i - c_j v_j into V_{j+1}.
__global__ void __launch_bounds__(kBlock) k_gm_update2(Batch bt, int tiles, size_t n, Gmres gm, int j,
                                                       double2* __restrict__ V, size_t vstride,
                                                       const double2* __restrict__ z, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const Slot& S = bt.slots[slot];
  if (S.status != kActive || S.phase != 0) return;
  const size_t base = (size_t)slot * stride;
  const double2* sv = gm.hc + (size_t)slot * 2 * (gm.m + 1);
  const double2* cv = sv + gm.m + 1;
  const double ir = 1.0 / S.scal.x;
  double2* uj = V + (size_t)j * vstride + base;
  double2* un = V + (size_t)(j + 1) * vstride + base;
  // basis vector by basis vector, the thread's kVecPerThread nodes of each in
  // flight together
  double2 av[kVecPerThread], au[kVecPerThread];
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    av[e] = i < n ? uj[i] : c2(0.0, 0.0);
    au[e] = i < n ? cscale(ir, z[base + i]) : c2(0.0, 0.0);
  }
  for (int q = 0; q < j; ++q) {
    const double2 sq = sv[q], cq = cv[q];
    const double2* vq = V + (size_t)q * vstride + base;
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e) {
      const size_t i = vec_index(tile, e);
      if (i < n) {
        const double2 x = vq[i];
        av[e] = csub(av[e], cmul(sq, x));
        au[e] = csub(au[e], cmul(cq, x));
      }
    }
  }
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) {
      const double2 vj = cscale(ir, av[e]);
      uj[i] = vj;
      un[i] = csub(au[e], cmul(cv[j], vj));
    }
  }
}

// y = H^-1 g (upper triangular, k = cyc_k), one thread per slot of the list.
__global__ void k_gm_solve(Batch bt, int cap, Gmres gm) {
  const int si = blockIdx.x * blockDim.x + threadIdx.x;
  if (si >= cap || si >= *bt.nactive) return;
  const int slot = bt.active[si];
  const Slot& S = bt.slots[slot];
  if (S.status != kActive) return;
  const int k = S.cyc_k, m1 = gm.m + 1;
  const double2* H = gm.H + (size_t)slot * m1 * gm.m;
  const double2* gg = gm.g + (size_t)slot * m1;
  double2* y = gm.y + (size_t)slot * gm.m;
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = gg[i];
    for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(H[(size_t)l * m1 + i], y[l]));
    y[i] = cdiv(acc, H[(size_t)i * m1 + i]);
  }
}

// t = sum_{i < cyc_k} y_i V_i
__global__ void __launch_bounds__(kBlock) k_gm_combine(Batch bt, int tiles, size_t n, Gmres gm,
                                                       const double2* __restrict__ V, size_t vstride,
                                                       double2* __restrict__ t, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
  const int k = bt.slots[slot].cyc_k;
  const double2* y = gm.y + (size_t)slot * gm.m;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) {
      double2 acc = c2(0.0, 0.0);
      for (int q = 0; q < k; ++q) acc = cadd(acc, cmul(y[q], V[(size_t)q * vstride + base + i]));
      t[base + i] = acc;
    }
  }
}

// x += z
__global__ void __launch_bounds__(kBlock) k_axpy1(Batch bt, int tiles, size_t n,
                                                  const double2* __restrict__ z,
                                                  double2* __restrict__ x, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = vec_index(tile, e);
    if (i < n) x[base + i] = cadd(x[base + i], z[base + i]);
  }
}

// ---------------------------------------------------------------- launchers
static inline dim3 grid1(long long blocks) { return dim3((unsigned)blocks); }

hipError_t launch_copy(const Batch& bt, int cap, size_t n, const double2* x, double2* y,
                       size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_copy, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, x, y, stride);
  return hipGetLastError();
}

hipError_t launch_repitch(int nslots, int nz, int nx, const double2* src, int sp, size_t ss, double2* dst, int dp,
                          size_t ds, hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  if (nz <= 0 || nx <= 0 || sp < nx || dp < nx || ss < (size_t)nz * sp || ds < (size_t)nz * dp || !src || !dst)
    return hipErrorInvalidValue;
  const size_t total = (size_t)nslots * nz * dp;
  hipLaunchKernelGGL(k_repitch, grid1((long long)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, nz, nx, src,
                     sp, ss, dst, dp, ds, total);
  return hipGetLastError();
}

hipError_t launch_bicg_init(size_t n, const Batch& bt, int cap, const Reduce& rd, const double2* b,
                            double2* x, double2* r, double2* rh, double2* p, double2* v,
                            size_t stride, hipStream_t st, size_t bstride, int nx, int px) {
  if (cap <= 0) return hipSuccess;
  if (px != 0 && (nx <= 0 || px < nx || n % (size_t)nx != 0 || stride < n / nx * px)) return hipErrorInvalidValue;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_init, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, rd, b, x, r, rh, p,
                     v, stride, bstride ? bstride : stride, nx, px);
  return hipGetLastError();
}

hipError_t launch_bicg_p(size_t n, const Batch& bt, int cap, const double2* r, const double2* p_old,
                         const double2* v, double2* p_new, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_p, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, r, p_old, v, p_new, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_apply_sigma(int dim, const Grid& g, const Batch& bt, int cap,
                                   const Reduce& rd, const double2* ph, const double2* rh,
                                   double2* v, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (!v && dim != 2) return hipErrorInvalidValue;
  if (dim == 3) {
    const Tiles t3 = grid_tiles(g.nz * g.ny, g.nx, 3);
    hipLaunchKernelGGL(k_bicg_apply3<0>, grid1(tile_blocks(t3.per_slot, cap)), dim3(kBlock), 0, st, g, t3, bt, rd,
                       ph, rh, v, stride);
    return hipGetLastError();
  }
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  if (dim == 2) {
    if (g.rho && !g.dc) return hipErrorInvalidValue;  // a density needs the level's coupling table
    const int ntx = (g.nx + kTX - 1) / kTX, per = lds_tiles(g.nz, g.nx);
    if (g.dc)
      hipLaunchKernelGGL((k_bicg_apply_t<0, true>), grid1(tile_blocks(per, cap)), dim3(kBlock), 0, st, g, ntx, per,
                         bt, rd, ph, rh, v, stride);
    else
      hipLaunchKernelGGL((k_bicg_apply_t<0, false>), grid1(tile_blocks(per, cap)), dim3(kBlock), 0, st, g, ntx, per,
                         bt, rd, ph, rh, v, stride);
  } else
    hipLaunchKernelGGL(k_bicg_apply_sigma<false>, gr, dim3(kBlock), 0, st, g, t, bt, rd, ph, rh, v, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_s(size_t n, const Batch& bt, int cap, const double2* r, const double2* v,
                         double2* s, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_s, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, r, v, s, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_apply_omega(int dim, const Grid& g, const Batch& bt, int cap,
                                   const Reduce& rd, const double2* sh, const double2* s,
                                   double2* t, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (!t && dim != 2) return hipErrorInvalidValue;
  if (dim == 3) {
    const Tiles t3 = grid_tiles(g.nz * g.ny, g.nx, 3);
    hipLaunchKernelGGL(k_bicg_apply3<1>, grid1(tile_blocks(t3.per_slot, cap)), dim3(kBlock), 0, st, g, t3, bt, rd,
                       sh, s, t, stride);
    return hipGetLastError();
  }
  const Tiles tl = grid_tiles(g.nz, g.nx, dim);
  const dim3 gr = grid1(tile_blocks(tl.per_slot, cap));
  if (dim == 2) {
    if (g.rho && !g.dc) return hipErrorInvalidValue;  // a density needs the level's coupling table
    const int ntx = (g.nx + kTX - 1) / kTX, per = lds_tiles(g.nz, g.nx);
    if (g.dc)
      hipLaunchKernelGGL((k_bicg_apply_t<1, true>), grid1(tile_blocks(per, cap)), dim3(kBlock), 0, st, g, ntx, per,
                         bt, rd, sh, s, t, stride);
    else
      hipLaunchKernelGGL((k_bicg_apply_t<1, false>), grid1(tile_blocks(per, cap)), dim3(kBlock), 0, st, g, ntx, per,
                         bt, rd, sh, s, t, stride);
  } else
    hipLaunchKernelGGL(k_bicg_apply_omega<false>, gr, dim3(kBlock), 0, st, g, tl, bt, rd, sh, s, t, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_xr(size_t n, const Batch& bt, int cap, const Reduce& rd, double2* x,
                          const double2* ph, const double2* sh, const double2* s, const double2* t,
                          double2* r, const double2* rh, size_t stride, hipStream_t st, int ring,
                          const double2* ph0, const double2* sh0) {
  if (cap <= 0) return hipSuccess;
  if (ring == 1 && (!ph0 || !sh0)) return hipErrorInvalidValue;
  const int tiles = vec_tiles(n);
  const dim3 gr = grid1((long long)cap * tiles);
  if (ring < 0)
    hipLaunchKernelGGL(k_bicg_xr<-1>, gr, dim3(kBlock), 0, st, bt, tiles, n, rd, x, ph, sh, ph0, sh0, s, t, r, rh,
                       stride);
  else if (ring == 0)
    hipLaunchKernelGGL(k_bicg_xr<0>, gr, dim3(kBlock), 0, st, bt, tiles, n, rd, x, ph, sh, ph0, sh0, s, t, r, rh,
                       stride);
  else
    hipLaunchKernelGGL(k_bicg_xr<1>, gr, dim3(kBlock), 0, st, bt, tiles, n, rd, x, ph, sh, ph0, sh0, s, t, r, rh,
                       stride);
  return hipGetLastError();
}

hipError_t launch_bicg_xr_t(const Grid& g, const Batch& bt, int cap, const Reduce& rd, double2* x,
                            const double2* ph, const double2* sh, const double2* s, double2* r,
                            const double2* rh, size_t stride, hipStream_t st, int ring, const double2* ph0,
                            const double2* sh0) {
  if (cap <= 0) return hipSuccess;
  if (ring == 1 && (!ph0 || !sh0)) return hipErrorInvalidValue;
  if (g.rho && !g.dc) return hipErrorInvalidValue;  // a density needs the level's coupling table
  if (stride < (size_t)g.nz * vpitch(g) || vpitch(g) < g.nx || ring < -1 || ring > 1) return hipErrorInvalidValue;
  const int ntx = (g.nx + kTX - 1) / kTX, per = lds_tiles(g.nz, g.nx);
  const dim3 gr = grid1(tile_blocks(per, cap));
#define HZ_XR_T(XM, RH)                                                                                          \
  hipLaunchKernelGGL((k_bicg_xr_t<XM, RH>), gr, dim3(kBlock), 0, st, g, ntx, per, bt, rd, x, ph, sh, ph0, sh0, s, \
                     r, rh, stride)
  const bool dc = g.dc != nullptr;
  if (ring < 0) {
    if (dc) HZ_XR_T(-1, true); else HZ_XR_T(-1, false);
  } else if (ring == 0) {
    if (dc) HZ_XR_T(0, true); else HZ_XR_T(0, false);
  } else {
    if (dc) HZ_XR_T(1, true); else HZ_XR_T(1, false);
  }
#undef HZ_XR_T
  return hipGetLastError();
}

hipError_t launch_bicg_flush(size_t n, int nslots, const Batch& bt, int only_restart, double2* x,
                             const double2* ph0, const double2* sh0, size_t stride, hipStream_t st, int slot0) {
  if (nslots <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_flush, grid1((long long)nslots * tiles), dim3(kBlock), 0, st, bt, tiles, n, only_restart,
                     x, ph0, sh0, stride, slot0);
  return hipGetLastError();
}

hipError_t launch_bicg_restart(size_t n, int nslots, const Batch& bt, const Reduce& rd,
                               const double2* r, double2* rh, double2* p, double2* v,
                               size_t stride, hipStream_t st, int nx, int px) {
  if (px != 0 && (nx <= 0 || px < nx || n % (size_t)nx != 0 || stride < n / nx * px)) return hipErrorInvalidValue;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_restart, grid1((long long)nslots * tiles), dim3(kBlock), 0, st, tiles, n, bt, rd, r, rh,
                     p, v, stride, nx, px);
  return hipGetLastError();
}

hipError_t launch_bicg_fin(int which, int tiles, const Batch& bt, int cap, const Reduce& rd,
                           double tol, int maxit, const double2* vec, size_t stride, hipStream_t st, int ring,
                           int restart_at, const Grid* g) {
  if (cap <= 0) return hipSuccess;
  if ((which == kFinSigma || which == kFinSigmaB || which == kFinStep) && !vec) return hipErrorInvalidValue;
  if (which == kFinSigmaB && !g) return hipErrorInvalidValue;
  const Grid gg = g ? *g : Grid{0, 0, 0.0, nullptr};
  hipLaunchKernelGGL(k_bicg_fin, dim3(cap), dim3(kBlock), 0, st, which, tiles, bt, rd, tol, maxit, vec, stride,
                     ring, restart_at, gg);
  return hipGetLastError();
}

hipError_t launch_rh_sparse(size_t n, int nslots, const Batch& bt, const double2* b, int* idx, double2* val,
                            size_t stride, hipStream_t st, int slot0) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rh_sparse, dim3(nslots), dim3(kBlock), 0, st, n, bt, b, idx, val, stride, slot0);
  return hipGetLastError();
}

hipError_t launch_compact(int nslots, int nrhs, int nfreq, Slot* slots, int* active, int* nactive,
                          int* fstart, Summary* sum, int want_phase, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, nslots, nrhs, nfreq, slots, active, nactive, fstart, sum, want_phase);
  return hipGetLastError();
}

hipError_t launch_true_residual(int dim, const Grid& g, const Batch& bt, int cap, const Reduce& rd,
                                const double2* b, const double2* x, double* out, size_t stride,
                                hipStream_t st) {
  const Tiles t = dim == 3 ? grid_tiles(g.nz * g.ny, g.nx, 3) : grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  if (dim == 3)
    hipLaunchKernelGGL(k_true_residual3, gr, dim3(kBlock), 0, st, g, t, bt, rd, b, x, stride);
  else if (dim == 2)
    hipLaunchKernelGGL(k_true_residual<true>, gr, dim3(kBlock), 0, st, g, t, bt, rd, b, x, stride);
  else
    hipLaunchKernelGGL(k_true_residual<false>, gr, dim3(kBlock), 0, st, g, t, bt, rd, b, x, stride);
  hipLaunchKernelGGL(k_true_residual_fin, dim3(cap), dim3(kBlock), 0, st, t.per_slot, bt, rd, out);
  return hipGetLastError();
}

hipError_t launch_gm_residual(int dim, const Grid& g, const Batch& bt, int cap, const Reduce& rd,
                              const Gmres& gm, int first, double tol, int maxit, const double2* b,
                              double2* x, double2* v0, size_t stride, hipStream_t st) {
  const Tiles t = dim == 3 ? grid_tiles(g.nz * g.ny, g.nx, 3) : grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  if (dim == 3)
    hipLaunchKernelGGL(k_gm_residual3, gr, dim3(kBlock), 0, st, g, t, bt, rd, first, b, x, v0, stride);
  else if (dim == 2)
    hipLaunchKernelGGL(k_gm_residual<true>, gr, dim3(kBlock), 0, st, g, t, bt, rd, first, b, x, v0, stride);
  else
    hipLaunchKernelGGL(k_gm_residual<false>, gr, dim3(kBlock), 0, st, g, t, bt, rd, first, b, x, v0, stride);
  hipLaunchKernelGGL(k_gm_residual_fin, dim3(cap), dim3(kBlock), 0, st, t.per_slot, bt, rd, gm, first, tol, maxit);
  return hipGetLastError();
}

hipError_t launch_gm_scale(size_t n, const Batch& bt, int cap, double2* v, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_gm_scale, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, v, stride);
  return hipGetLastError();
}

int gm_dot_tiles(size_t n) { return (int)((n + kGmDotNodes - 1) / kGmDotNodes); }

hipError_t launch_gm_step(size_t n, const Batch& bt, int cap, const Gmres& gm, int j, int finish, double tol,
                          int maxit, double2* V, size_t vstride, const double2* z, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (finish ? z != nullptr : z == nullptr) return hipErrorInvalidValue;
  const int tiles = vec_tiles(n);
  const int dtiles = gm_dot_tiles(n);
  if (dtiles > gm.max_tiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gm_dots2, grid1((long long)cap * dtiles), dim3(kBlock),
                     (size_t)kWaves * (4 * j + 3) * sizeof(double), st, bt, dtiles, n, gm, j, V, vstride, z, stride);
  const size_t fin_lds = (size_t)((4 * j + 4) & ~1) * sizeof(double) + (size_t)(j + 1) * sizeof(double2) +
                         2 * sizeof(double);
  hipLaunchKernelGGL(k_gm_fin2, dim3(cap), dim3(kBlock), fin_lds, st, dtiles, bt, gm, j, tol, maxit, finish);
  if (!finish)
    hipLaunchKernelGGL(k_gm_update2, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, gm, j, V,
                       vstride, z, stride);
  return hipGetLastError();
}

hipError_t launch_gm_solve(const Batch& bt, int cap, const Gmres& gm, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gm_solve, dim3((cap + 63) / 64), dim3(64), 0, st, bt, cap, gm);
  return hipGetLastError();
}

hipError_t launch_gm_combine(size_t n, const Batch& bt, int cap, const Gmres& gm, const double2* V,
                             size_t vstride, double2* t, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_gm_combine, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, gm, V, vstride, t, stride);
  return hipGetLastError();
}

hipError_t launch_axpy1(size_t n, const Batch& bt, int cap, const double2* z, double2* x, size_t stride,
                        hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_axpy1, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, z, x, stride);
  return hipGetLastError();
}

}  // namespace hz
