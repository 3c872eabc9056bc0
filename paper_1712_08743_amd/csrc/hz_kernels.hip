// HIP kernels for gfx950 (MI355X): the complex128 Helmholtz stencil, the
// multigrid smoother and transfers, the coarse solve, the 1D tridiagonal
// solve, the batched BiCGSTAB updates with deterministic per-slot reductions,
// and the misfit pieces.
//
// Operator (Kazemi, arXiv:1712.08743, Eq. (2)-(3) with the first-order
// absorbing boundary of Eq. (1)), in weighted form, at node p = (iz, ix):
//   (A x)_p = [lsum_p x_p - wz (x_left + x_right) - wx (x_up + x_down)] / h^2
//             + kap_p x_p,
//   kap_p   = j omega g_p m_p / h - omega^2 s w_p m_p^2,
// wx, wz = 1/2 on end nodes of their axis (else 1), w = wx wz, g sums the
// other-axis weight over the axes on which p is an end node, lsum sums the
// couplings of the existing neighbours. s = 1 - j alpha gives B, s = beta1 -
// j beta2 the shifted Laplacian M. Missing neighbours contribute nothing.
//
// Every kernel is memory-bound (well under one flop per byte): the layouts
// are x-fastest complex128 rows read as 16-byte vectors by 64-wide
// wavefronts, one block per (slot, tile), with the slot list compacted on
// the device so that converged right-hand sides cost no launch slots.

#include "hz_device.h"
#include "hz_node3.h"

#include <math.h>

namespace hz {

// ---------------------------------------------------------------- grid geometry
Tiles grid_tiles(int nz, int nx, int dim) {
  Tiles t;
  if (dim == 3) {
    // 3D (nz counts the nz * ny rows): kBlock consecutive nodes per tile in
    // flat order (node3_of), so no thread idles at the end of a row
    t.tx = t.tz = t.ntx = t.ntz = 0;
    t.per_slot = (int)(((size_t)nz * nx + kBlock - 1) / kBlock);
    return t;
  }
  if (dim == 1) {
    t.tx = kBlock;
    t.tz = 1;
  } else {
    t.tx = 64;
    t.tz = kBlock / 64;
  }
  t.ntx = (nx + t.tx - 1) / t.tx;
  t.ntz = (nz + t.tz - 1) / t.tz;
  t.per_slot = t.ntx * t.ntz;
  return t;
}

long long tile_blocks(int per_slot, int cap) { return (long long)kXcd * xcd_chunk(per_slot) * cap; }

int lds_tiles(int nz, int nx) { return ((nx + kTX - 1) / kTX) * ((nz + kTZ - 1) / kTZ); }

int reduce_tiles(int nz, int nx, int dim) {
  return dim == 2 ? lds_tiles(nz, nx) : grid_tiles(nz, nx, dim).per_slot;
}

int vec_tiles(size_t n) {
  const size_t per = (size_t)kBlock * kVecPerThread;
  return (int)((n + per - 1) / per);
}

// ---------------------------------------------------------------- stencil kernels
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_apply(Grid g, Tiles t, int lvl, int which, Batch bt,
                                                  const double2* __restrict__ x,
                                                  double2* __restrict__ y, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= g.nz || ix >= g.nx) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double sre = which ? f.sM_re : f.sB_re, sim = which ? f.sM_im : f.sB_im;
  const int p = iz * g.nx + ix;
  const NodeOp o = node_op<D2>(g, iz, ix, p, model_m(g, f)[p], f.omega, sre, sim);
  const double2* xs = x + (size_t)slot * stride;
  y[(size_t)slot * stride + p] = apply_op<D2>(g, o, xs, p, iz, ix, 1.0 / (g.h * g.h), xs[p]);
  (void)lvl;
}

// u_out = u_in + w (b - M u_in) / diag(M); ZERO: u_in = 0.
// coarse_only: only slots whose frequency smooths its coarsest level
template <bool D2, bool ZERO>
__global__ void __launch_bounds__(kBlock) k_smooth(Grid g, Tiles t, int lvl, double w_override,
                                                   Batch bt, const double2* __restrict__ b,
                                                   const double2* __restrict__ u_in,
                                                   double2* __restrict__ u_out, size_t stride, int coarse_only) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= g.nz || ix >= g.nx) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  if (coarse_only && !f.coarse_jacobi) return;
  const int p = iz * g.nx + ix;
  const double ih2 = 1.0 / (g.h * g.h);
  const NodeOp o = node_op<D2>(g, iz, ix, p, model_m(g, f)[p], f.omega, f.sM_re, f.sM_im);
  // w / diag(M): tabulated per frequency and level, or formed here for an explicit weight
  const double2 wdinv = w_override > 0.0 ? cscale(w_override, cinv(diag_of<D2>(o.c, ih2))) : f.winv[lvl][p];
  const size_t base = (size_t)slot * stride;
  const double2 bp = b[base + p];
  double2 out;
  if (ZERO) {
    out = cmul(bp, wdinv);
  } else {
    const double2* us = u_in + base;
    const double2 up = us[p];
    const double2 res = csub(bp, apply_op<D2>(g, o, us, p, iz, ix, ih2, up));
    out = cadd(up, cmul(res, wdinv));
  }
  u_out[base + p] = out;
}

// winv[p] = w / diag(M)[p] on one level for one frequency.
template <bool D2>
__global__ void k_winv(Grid g, double omega, double s_re, double s_im, double w, double2* __restrict__ winv) {
  const size_t n = (size_t)g.nz * g.nx;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int iz = D2 ? (int)(p / g.nx) : 0;
  const int ix = (int)(p - (size_t)iz * g.nx);
  const NodeOp o = node_op<D2>(g, iz, ix, (int)p, g.m[p], omega, s_re, s_im);
  winv[p] = cscale(w, cinv(diag_of<D2>(o.c, 1.0 / (g.h * g.h))));
}

// bc = 2^-dim P^T (b - M u), one thread per coarse node. P^T gives the two
// fine neighbours of a coarse node weight 1/2, except the last fine node of
// an axis with an even node count, which is interpolated from the last coarse
// node alone and so carries weight 1 (coarse node J with 2J + 2 == n).
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_restrict(Grid gf, Grid gc, Tiles t, Batch bt,
                                                     const double2* __restrict__ b,
                                                     const double2* __restrict__ u,
                                                     double2* __restrict__ bc, size_t sf,
                                                     size_t sc) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int Iz, Ix;
  tile_node<D2>(t, tile, Iz, Ix);
  if (Iz >= gc.nz || Ix >= gc.nx) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double ih2 = 1.0 / (gf.h * gf.h);
  const double2* bs = b + (size_t)slot * sf;
  const double2* us = u + (size_t)slot * sf;
  double2 acc = c2(0.0, 0.0);
  const int dz_lo = D2 ? -1 : 0, dz_hi = D2 ? 1 : 0;
  for (int dz = dz_lo; dz <= dz_hi; ++dz) {
    const int iz = D2 ? 2 * Iz + dz : 0;
    if (iz < 0 || iz >= gf.nz) continue;
    const double wzt = (dz == 0 || (dz == 1 && 2 * Iz + 2 == gf.nz)) ? 1.0 : 0.5;
    double2 row = c2(0.0, 0.0);
    for (int dx = -1; dx <= 1; ++dx) {
      const int ix = 2 * Ix + dx;
      if (ix < 0 || ix >= gf.nx) continue;
      const int p = iz * gf.nx + ix;
      const NodeOp o = node_op<D2>(gf, iz, ix, p, model_m(gf, f)[p], f.omega, f.sM_re, f.sM_im);
      const double2 r = csub(bs[p], apply_op<D2>(gf, o, us, p, iz, ix, ih2, us[p]));
      const double wxt = (dx == 0 || (dx == 1 && 2 * Ix + 2 == gf.nx)) ? 1.0 : 0.5;
      row = cadd(row, cscale(wxt, r));
    }
    acc = cadd(acc, cscale(wzt, row));
  }
  bc[(size_t)slot * sc + Iz * gc.nx + Ix] = cscale(D2 ? 0.25 : 0.5, acc);
}

// Bilinear (1D: linear) interpolation of coarse e at fine node (iz, ix). The
// last node of an even-count axis has no right coarse neighbour: the clamped
// index makes it (e_J + e_J) / 2 = e_J exactly.
template <bool D2>
__device__ __forceinline__ double2 interp(const double2* __restrict__ e, int iz, int ix, int ncx, int ncz) {
  const int Jx = ix >> 1, ox = ix & 1, Jx1 = min(Jx + 1, ncx - 1);
  if (!D2) {
    return ox ? cscale(0.5, cadd(e[Jx], e[Jx1])) : e[Jx];
  }
  const int Jz = iz >> 1, oz = iz & 1;
  const double2* r0 = e + Jz * ncx;
  double2 a = ox ? cscale(0.5, cadd(r0[Jx], r0[Jx1])) : r0[Jx];
  if (!oz) return a;
  const double2* r1 = Jz + 1 < ncz ? r0 + ncx : r0;
  const double2 bb = ox ? cscale(0.5, cadd(r1[Jx], r1[Jx1])) : r1[Jx];
  return cscale(0.5, cadd(a, bb));
}

// u_out = u_in + P e (u_out may be u_in: each thread reads, then writes, its own node).
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_prolong(Grid gf, Grid gc, Tiles t, Batch bt,
                                                    const double2* __restrict__ e,
                                                    const double2* u_in, double2* u_out,
                                                    size_t sf, size_t sc) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= gf.nz || ix >= gf.nx) return;
  const size_t q = (size_t)slot * sf + iz * gf.nx + ix;
  const double2 ef = interp<D2>(e + (size_t)slot * sc, iz, ix, gc.nx, gc.nz);
  u_out[q] = cadd(u_in[q], ef);
}

// ---------------------------------------------------------------- fused multigrid kernels
// Two damped-Jacobi sweeps from u = 0 in one pass: u1 = w b / D is formed at
// the node and its neighbours, then u2 = u1 + w (b - M u1) / D. MODE 1/2 also
// store the Krylov vector they form (into a buffer other than its inputs).
// Reads b's inputs at five nodes (neighbours come from cache), writes u2.
template <bool D2, int MODE>
__global__ void __launch_bounds__(kBlock) k_pre2(Grid g, Tiles t, int lvl, Batch bt, RhsIn in,
                                                 double2* __restrict__ bout,
                                                 double2* __restrict__ u2, size_t stride) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= g.nz || ix >= g.nx) return;
  const Slot& S = bt.slots[slot];
  const FreqTab& f = bt.ft[S.freq];
  double2 beta = c2(0.0, 0.0), om = c2(0.0, 0.0), al = c2(0.0, 0.0);
  if (MODE == 1) {
    beta = S.beta;
    om = S.omega;
  }
  if (MODE == 2) al = S.alpha;
  const double ih2 = 1.0 / (g.h * g.h);
  const size_t base = (size_t)slot * stride;
  const int p = iz * g.nx + ix;
  const double2* wd = f.winv[lvl];
  // u1 at a node q: (w / D_q) b_q
  auto u1_at = [&](int q) -> double2 { return cmul(rhs_at<MODE>(in, base + q, beta, om, al), wd[q]); };
  const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, 1.0 / g.h, model_m(g, f)[p], f.omega, f.sM_re, f.sM_im);
  const double2 wdp = wd[p];
  const double2 bp = rhs_at<MODE>(in, base + p, beta, om, al);
  const double2 u1p = cmul(bp, wdp);
  double2 sx = c2(0.0, 0.0), sz = c2(0.0, 0.0);
  if (ix > 0) sx = cadd(sx, u1_at(p - 1));
  if (ix < g.nx - 1) sx = cadd(sx, u1_at(p + 1));
  if (D2) {
    if (iz > 0) sz = cadd(sz, u1_at(p - g.nx));
    if (iz < g.nz - 1) sz = cadd(sz, u1_at(p + g.nx));
  }
  const double2 res = csub(bp, stencil(c, ih2, u1p, sx, sz));
  u2[base + p] = cadd(u1p, cmul(res, wdp));
  if (MODE != 0) bout[base + p] = bp;
}

// Prolongation, correction and one damped-Jacobi sweep in one pass:
// u3 = u2 + P e at the node and its neighbours, u_out = u3 + w (b - M u3) / D.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_prolong_smooth(Grid gf, Grid gc, Tiles t, int lvl, Batch bt,
                                                           const double2* __restrict__ e,
                                                           const double2* __restrict__ b,
                                                           const double2* __restrict__ u2,
                                                           double2* __restrict__ u_out, size_t sf,
                                                           size_t sc) {
  int slot, tile;
  if (!decode_tile(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= gf.nz || ix >= gf.nx) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double ih2 = 1.0 / (gf.h * gf.h);
  const size_t base = (size_t)slot * sf;
  const double2* es = e + (size_t)slot * sc;
  const double2* us = u2 + base;
  auto u3_at = [&](int qz, int qx) -> double2 {
    return cadd(us[qz * gf.nx + qx], interp<D2>(es, qz, qx, gc.nx, gc.nz));
  };
  const int p = iz * gf.nx + ix;
  const NodeOp o = node_op<D2>(gf, iz, ix, p, model_m(gf, f)[p], f.omega, f.sM_re, f.sM_im);
  const double2 u3p = u3_at(iz, ix);
  const double2 res = csub(b[base + p], apply_op_at<D2>(gf, o, iz, ix, ih2, u3p, [&](int dz, int dx) {
                             return u3_at(iz + dz, ix + dx);
                           }));
  u_out[base + p] = cadd(u3p, cmul(res, f.winv[lvl][p]));
}

// ---- LDS-tiled forms of the three smoothing kernels (2D grids)

// One sweep from a nonzero start, u staged in LDS.
__global__ void __launch_bounds__(kBlock) k_smooth_t(Grid g, int ntx, int per_slot, int lvl, Batch bt,
                                                     const double2* __restrict__ b,
                                                     const double2* __restrict__ u_in,
                                                     double2* __restrict__ u_out, size_t stride) {
  __shared__ double2 U[kHZ][kHX];
  int slot, tile;
  if (!decode_tile(bt, per_slot, slot, tile)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const TileOrg t = tile_org(tile, ntx);
  const size_t base = (size_t)slot * stride;
  const double2* us = u_in + base;
  fill_halo(U, g, t, [&](int q, int, int) { return us[q]; });
  __syncthreads();
  const double ih = 1.0 / g.h, ih2 = ih * ih;
  const double2* wd = f.winv[lvl];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int lz = threadIdx.x / kTX + (kBlock / kTX) * r, lx = threadIdx.x % kTX;
    const int iz = t.z0 + lz, ix = t.x0 + lx;
    if (iz >= g.nz || ix >= g.nx) continue;
    const int p = iz * g.nx + ix;
    const NodeC c = node_coef<true>(iz, ix, g.nz, g.nx, ih, model_m(g, f)[p], f.omega, f.sM_re, f.sM_im);
    double2 sx, sz;
    halo_sums(U, lz, lx, sx, sz);
    const double2 up = U[lz + 1][lx + 1];
    const double2 res = csub(b[base + p], stencil(c, ih2, up, sx, sz));
    u_out[base + p] = cadd(up, cmul(res, wd[p]));
  }
}

// Prolongation + correction + one sweep, u3 = u2 + P e staged in LDS.
__global__ void __launch_bounds__(kBlock) k_prolong_smooth_t(Grid gf, Grid gc, int ntx, int per_slot, int lvl,
                                                             Batch bt, const double2* __restrict__ e,
                                                             const double2* __restrict__ b,
                                                             const double2* __restrict__ u2,
                                                             double2* __restrict__ u_out, size_t sf,
                                                             size_t sc) {
  __shared__ double2 U[kHZ][kHX];
  int slot, tile;
  if (!decode_tile(bt, per_slot, slot, tile)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const TileOrg t = tile_org(tile, ntx);
  const size_t base = (size_t)slot * sf;
  const double2* us = u2 + base;
  const double2* es = e + (size_t)slot * sc;
  fill_halo(U, gf, t, [&](int q, int hz, int hx) {
    const int qz = t.z0 - 1 + hz, qx = t.x0 - 1 + hx;
    return cadd(us[q], interp<true>(es, qz, qx, gc.nx, gc.nz));
  });
  __syncthreads();
  const double ih = 1.0 / gf.h, ih2 = ih * ih;
  const double2* wd = f.winv[lvl];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int lz = threadIdx.x / kTX + (kBlock / kTX) * r, lx = threadIdx.x % kTX;
    const int iz = t.z0 + lz, ix = t.x0 + lx;
    if (iz >= gf.nz || ix >= gf.nx) continue;
    const int p = iz * gf.nx + ix;
    const NodeC c = node_coef<true>(iz, ix, gf.nz, gf.nx, ih, model_m(gf, f)[p], f.omega, f.sM_re, f.sM_im);
    double2 sx, sz;
    halo_sums(U, lz, lx, sx, sz);
    const double2 u3p = U[lz + 1][lx + 1];
    const double2 res = csub(b[base + p], stencil(c, ih2, u3p, sx, sz));
    u_out[base + p] = cadd(u3p, cmul(res, wd[p]));
  }
}

// Weighted-residual restriction with the fine residual computed once per
// fine node in LDS. A block owns a kRtz x kRtx tile of coarse nodes; it loads
// u on the covering fine region plus a one-node halo, forms r = b - M u on the
// region (fine nodes 2I-1 .. 2I+1 of every coarse node I), then takes the
// 3 x 3 full-weighting sum (times 1/4) per coarse node.
constexpr int kRtx = 32, kRtz = 8;
constexpr int kRfx = 2 * kRtx + 1, kRfz = 2 * kRtz + 1;  // residual region
constexpr int kRux = kRfx + 2, kRuz = kRfz + 2;          // u region (halo 1)

__global__ void __launch_bounds__(kRtx * kRtz) k_restrict_tiled(Grid gf, Grid gc, int ntx, int per_slot,
                                                                Batch bt, const double2* __restrict__ b,
                                                                const double2* __restrict__ u,
                                                                double2* __restrict__ bc, size_t sf,
                                                                size_t sc) {
  __shared__ double2 U[kRuz][kRux];
  __shared__ double2 Rr[kRfz][kRfx];
  int slot, tile;
  if (!decode_tile(bt, per_slot, slot, tile)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const int tzi = tile / ntx, txi = tile - tzi * ntx;
  const int cz0 = tzi * kRtz, cx0 = txi * kRtx;
  const int fz0 = 2 * cz0 - 1, fx0 = 2 * cx0 - 1;  // fine origin of the residual region
  const size_t base = (size_t)slot * sf;
  const double2* us = u + base;
  const double2* bs = b + base;
  for (int e = threadIdx.x; e < kRuz * kRux; e += blockDim.x) {
    const int lz = e / kRux, lx = e - lz * kRux;
    const int gz = fz0 - 1 + lz, gx = fx0 - 1 + lx;
    U[lz][lx] = (gz >= 0 && gz < gf.nz && gx >= 0 && gx < gf.nx) ? us[gz * gf.nx + gx] : c2(0.0, 0.0);
  }
  __syncthreads();
  const double ih2 = 1.0 / (gf.h * gf.h);
  for (int e = threadIdx.x; e < kRfz * kRfx; e += blockDim.x) {
    const int lz = e / kRfx, lx = e - lz * kRfx;
    const int iz = fz0 + lz, ix = fx0 + lx;
    double2 r = c2(0.0, 0.0);
    if (iz >= 0 && iz < gf.nz && ix >= 0 && ix < gf.nx) {
      const int p = iz * gf.nx + ix;
      const NodeC c = node_coef<true>(iz, ix, gf.nz, gf.nx, 1.0 / gf.h, model_m(gf, f)[p], f.omega, f.sM_re, f.sM_im);
      const int uz = lz + 1, ux = lx + 1;
      double2 sx = c2(0.0, 0.0), sz = c2(0.0, 0.0);
      if (ix > 0) sx = cadd(sx, U[uz][ux - 1]);
      if (ix < gf.nx - 1) sx = cadd(sx, U[uz][ux + 1]);
      if (iz > 0) sz = cadd(sz, U[uz - 1][ux]);
      if (iz < gf.nz - 1) sz = cadd(sz, U[uz + 1][ux]);
      r = csub(bs[p], stencil(c, ih2, U[uz][ux], sx, sz));
    }
    Rr[lz][lx] = r;
  }
  __syncthreads();
  const int lcz = threadIdx.x / kRtx, lcx = threadIdx.x - lcz * kRtx;
  const int Iz = cz0 + lcz, Ix = cx0 + lcx;
  if (Iz >= gc.nz || Ix >= gc.nx) return;
  // residual-region index of fine node 2I + d is 2 * local + 1 + d
  const int rz = 2 * lcz + 1, rx = 2 * lcx + 1;
  // the last fine node of an even-count axis carries weight 1 (see k_restrict)
  const bool xe = 2 * Ix + 2 == gf.nx, ze = 2 * Iz + 2 == gf.nz;
  double2 acc = c2(0.0, 0.0);
  for (int dz = -1; dz <= 1; ++dz) {
    const double wzt = (dz == 0 || (dz == 1 && ze)) ? 1.0 : 0.5;
    const double2* R = Rr[rz + dz];
    const double2 row = xe ? cadd(cadd(R[rx], cscale(0.5, R[rx - 1])), R[rx + 1])
                           : cadd(R[rx], cscale(0.5, cadd(R[rx - 1], R[rx + 1])));
    acc = cadd(acc, cscale(wzt, row));
  }
  bc[(size_t)slot * sc + Iz * gc.nx + Ix] = cscale(0.25, acc);
}

// ---------------------------------------------------------------- coarse solve
// uc[slot] = Cinv_f bc[slot] for every active slot: per frequency a dense
// (nc x nc) by (nc x slots) complex product, on the matrix cores. A wave
// owns a 16-row by 16-slot tile and steps through K four columns at a time
// with v_mfma_f64_16x16x4f64, forming the complex product from four real
// ones: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br. Cinv is symmetric (M is
// complex symmetric), so the A operand (row r, column k) is read as
// Cinv[k][r]: 16 consecutive entries per k. Operand layout of the
// instruction: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and
// D[i][j] in lane j + 16 (i % 4), register i / 4. Grid: x = groups of
// kCoarseWaves row tiles, y = tiles of 16 active slots, z = frequency.
// Each output is a fixed-order sum over K for its own slot, so results do
// not depend on which other slots share the tile.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kCoarseWaves * 64) k_coarse(int nc, Batch bt,
                                                              const double2* __restrict__ bc,
                                                              double2* __restrict__ uc, size_t stride) {
  const int f = blockIdx.z;
  if (bt.ft[f].coarse_jacobi) return;  // that frequency's coarsest level is smoothed instead
  const int lo = bt.fstart[f], hi = bt.fstart[f + 1];
  const int s0 = lo + blockIdx.y * 16;
  if (s0 >= hi) return;  // uniform over the block
  const int lane = threadIdx.x & 63;
  const int r0 = (blockIdx.x * kCoarseWaves + (int)(threadIdx.x >> 6)) * 16;
  if (r0 >= nc) return;  // uniform over the wave
  const int i = lane & 15, kq = lane >> 4;
  const int row = min(r0 + i, nc - 1);  // rows past nc give outputs that are not stored
  const int slot = s0 + i < hi ? bt.active[s0 + i] : -1;
  const double2* Ci = bt.ft[f].cinv;
  const double2* bs = bc + (size_t)(slot < 0 ? 0 : slot) * stride;
  v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
  // columns of a slot past the active list read slot 0's data: MFMA columns
  // are independent and those outputs are never stored
  auto step = [&](double2 a, double2 b) {
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
  };
  const int kfull = nc & ~3;
  constexpr int kU = 8;  // K steps whose operands are loaded together
  int k0 = 0;
  for (; k0 + 4 * kU <= kfull; k0 += 4 * kU) {
    double2 a[kU], b[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + 4 * u + kq;
      a[u] = Ci[(size_t)k * nc + row];
      b[u] = bs[k];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) step(a[u], b[u]);
  }
  for (; k0 < kfull; k0 += 4) {
    const int k = k0 + kq;
    step(Ci[(size_t)k * nc + row], bs[k]);
  }
  if (kfull < nc) {  // last partial step: columns past nc contribute zero
    const int k = kfull + kq;
    const bool ok = k < nc;
    const int kk = ok ? k : nc - 1;
    const double2 a = Ci[(size_t)kk * nc + row], b = bs[kk];
    step(c2(ok ? a.x : 0.0, ok ? a.y : 0.0), c2(ok ? b.x : 0.0, ok ? b.y : 0.0));
  }
  const int j = lane & 15, i0 = lane >> 4;
  if (s0 + j >= hi) return;
  const int sl = bt.active[s0 + j];
  double2* us = uc + (size_t)sl * stride;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r0 + i0 + 4 * r < nc) us[r0 + i0 + 4 * r] = c2(cr[r], ci[r]);
}

// Dense M on the coarsest grid for every frequency: A[f][i][j].
template <bool D2>
__global__ void k_assemble_dense(Grid g, int nfreq, const FreqTab* __restrict__ ft,
                                 double2* __restrict__ A) {
  const size_t nc = (size_t)g.nz * g.nx;
  const size_t total = nc * nc * nfreq;
  const double ih2 = 1.0 / (g.h * g.h);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int f = (int)(e / (nc * nc));
    const size_t rem = e - (size_t)f * nc * nc;
    const int i = (int)(rem / nc), j = (int)(rem - (size_t)i * nc);
    const int iz = i / g.nx, ix = i - iz * g.nx;
    const int jz = j / g.nx, jx = j - jz * g.nx;
    const NodeOp o = node_op<D2>(g, iz, ix, i, model_m(g, ft[f])[i], ft[f].omega, ft[f].sM_re, ft[f].sM_im);
    const NodeC& c = o.c;
    double2 val = c2(0.0, 0.0);
    if (i == j) {
      val = diag_of<D2>(c, ih2);
    } else if (jz == iz && (jx == ix - 1 || jx == ix + 1)) {
      val = c2(-(g.rho ? o.cq[jx == ix - 1 ? 0 : 1] : c.wz) * ih2, 0.0);
    } else if (D2 && jx == ix && (jz == iz - 1 || jz == iz + 1)) {
      val = c2(-(g.rho ? o.cq[jz == iz - 1 ? 2 : 3] : c.wx) * ih2, 0.0);
    }
    A[e] = val;
  }
}

// One Gauss-Jordan pivot step on column k (no pivoting: M has a positive
// definite imaginary part, so every leading block is nonsingular).
__global__ void k_gj_step(int nc, int nfreq, int k, const double2* __restrict__ Ain,
                          double2* __restrict__ Aout) {
  const size_t n2 = (size_t)nc * nc;
  const size_t total = n2 * nfreq;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t f = e / n2;
    const size_t rem = e - f * n2;
    const int i = (int)(rem / nc), j = (int)(rem - (size_t)i * nc);
    const double2* A = Ain + f * n2;
    const double2 piv = cinv(A[(size_t)k * nc + k]);
    double2 out;
    if (i == k && j == k) {
      out = piv;
    } else if (i == k) {
      out = cmul(A[(size_t)k * nc + j], piv);
    } else if (j == k) {
      const double2 t = cmul(A[(size_t)i * nc + k], piv);
      out = c2(-t.x, -t.y);
    } else {
      out = csub(A[rem], cmul(cmul(A[(size_t)i * nc + k], piv), A[(size_t)k * nc + j]));
    }
    Aout[e] = out;
  }
}

// ---------------------------------------------------------------- 1D exact solve
// Parallel cyclic reduction of the tridiagonal M in LDS, one block per slot.
__global__ void __launch_bounds__(1024) k_pcr(Grid g, Batch bt, const double2* __restrict__ b,
                                              double2* __restrict__ u, size_t stride) {
  extern __shared__ double2 lds[];
  const int si = blockIdx.x;
  if (si >= *bt.nactive) return;
  const int slot = bt.active[si];
  if (bt.slots[slot].status != kActive) return;
  const int n = g.nx;
  double2* A = lds;
  double2* Bd = lds + n;
  double2* Cu = lds + 2 * n;
  double2* D = lds + 3 * n;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double ih2 = 1.0 / (g.h * g.h);
  const double2* bs = b + (size_t)slot * stride;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const NodeOp o = node_op<false>(g, 0, i, i, model_m(g, f)[i], f.omega, f.sM_re, f.sM_im);
    A[i] = c2(i > 0 ? -(g.rho ? o.cq[0] : 1.0) * ih2 : 0.0, 0.0);
    Cu[i] = c2(i < n - 1 ? -(g.rho ? o.cq[1] : 1.0) * ih2 : 0.0, 0.0);
    Bd[i] = diag_of<false>(o.c, ih2);
    D[i] = bs[i];
  }
  __syncthreads();
  constexpr int E = kPcrMax / 1024;
  for (int s = 1; s < n; s <<= 1) {
    double2 na[E], nb[E], ncu[E], nd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = threadIdx.x + e * 1024;
      if (i >= n) continue;
      double2 ai = A[i], bi = Bd[i], ci = Cu[i], di = D[i];
      double2 ra = c2(0.0, 0.0), rc = c2(0.0, 0.0);
      if (i - s >= 0) {
        const double2 k1 = cdiv(ai, Bd[i - s]);
        ra = cmul(k1, A[i - s]);
        bi = csub(bi, cmul(k1, Cu[i - s]));
        di = csub(di, cmul(k1, D[i - s]));
      }
      if (i + s < n) {
        const double2 k2 = cdiv(ci, Bd[i + s]);
        rc = cmul(k2, Cu[i + s]);
        bi = csub(bi, cmul(k2, A[i + s]));
        di = csub(di, cmul(k2, D[i + s]));
      }
      na[e] = c2(-ra.x, -ra.y);
      ncu[e] = c2(-rc.x, -rc.y);
      nb[e] = bi;
      nd[e] = di;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = threadIdx.x + e * 1024;
      if (i >= n) continue;
      A[i] = na[e];
      Bd[i] = nb[e];
      Cu[i] = ncu[e];
      D[i] = nd[e];
    }
    __syncthreads();
  }
  double2* us = u + (size_t)slot * stride;
  for (int i = threadIdx.x; i < n; i += blockDim.x) us[i] = cdiv(D[i], Bd[i]);
}

// ---------------------------------------------------------------- misfit, sources, model
__global__ void k_point_rhs_zero(size_t total, double2* __restrict__ b) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = c2(0.0, 0.0);
}

__global__ void k_point_rhs_set(size_t n, int nsrc, const int* __restrict__ nodes,
                                const double2* __restrict__ amp, double scale,
                                double2* __restrict__ b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsrc) return;
  const double2 a = amp ? amp[s] : c2(1.0, 0.0);
  b[(size_t)s * n + nodes[s]] = cscale(scale, a);
}

__global__ void k_gather(int nrhs, int nrec, const int* __restrict__ rec, const double2* __restrict__ u,
                         size_t stride, double2* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrhs * nrec) return;
  const int s = i / nrec, r = i - s * nrec;
  d[i] = u[(size_t)s * stride + rec[r]];
}

// out[0] = sum |d_obs - d_cal|^2 + lambda sum m^2 (one block, fixed order).
__global__ void __launch_bounds__(1024) k_misfit(size_t nd, const double2* __restrict__ dobs,
                                                 const double2* __restrict__ dcal, size_t nm,
                                                 const double* __restrict__ m, double lambda,
                                                 double* __restrict__ out) {
  __shared__ double sh[2][16];
  double a = 0.0, b = 0.0;
  for (size_t i = threadIdx.x; i < nd; i += blockDim.x) {
    const double2 e = csub(dobs[i], dcal[i]);
    a += e.x * e.x + e.y * e.y;
  }
  for (size_t i = threadIdx.x; i < nm; i += blockDim.x) b += m[i] * m[i];
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wid] = a;
    sh[1][wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      sa += sh[0][w];
      sb += sh[1][w];
    }
    out[0] = sa + lambda * sb;
    out[1] = sa;
    out[2] = sb;
  }
}

__global__ void k_inject(Grid gf, int dim, double* __restrict__ mc) {
  const int ncx = (gf.nx + 1) / 2;
  const int ncz = dim == 2 ? (gf.nz + 1) / 2 : 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncx * ncz) return;
  const int Iz = i / ncx, Ix = i - Iz * ncx;
  const int fz = dim == 2 ? 2 * Iz : 0;
  mc[i] = gf.m[(size_t)fz * gf.nx + 2 * Ix];
}

// out3 = {min m, max m, count of entries that are not finite and positive}
__global__ void __launch_bounds__(1024) k_check_model(size_t n, const double* __restrict__ m,
                                                      double* __restrict__ out3) {
  __shared__ double sh[3][16];
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = m[i];
    if (!(isfinite(v) && v > 0.0)) {
      bad += 1.0;
    } else {
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    bad += __shfl_xor(bad, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wid] = lo;
    sh[1][wid] = hi;
    sh[2][wid] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      sh[0][0] = fmin(sh[0][0], sh[0][w]);
      sh[1][0] = fmax(sh[1][0], sh[1][w]);
      sh[2][0] += sh[2][w];
    }
    out3[0] = sh[0][0];
    out3[1] = sh[1][0];
    out3[2] = sh[2][0];
  }
}

// The coupling table of a 2D level with a density (see RhoC): for node (iz, ix)
// wz (rho_p + rho_right) / 2 (zero on the last column), wx (rho_p + rho_below)
// / 2 (zero on the last row) and g sqrt(rho_p), the same values node_op forms.
__global__ void k_density_coef(Grid g, double* __restrict__ dc) {
  const size_t n = (size_t)g.nz * g.nx;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int iz = (int)(p / g.nx), ix = (int)(p - (size_t)iz * g.nx);
  const double* r = g.rho;
  const double rp = r[p];
  const int x0 = ix == 0, x1 = ix == g.nx - 1, z0 = iz == 0, z1 = iz == g.nz - 1;
  const double wx = (x0 | x1) ? 0.5 : 1.0, wz = (z0 | z1) ? 0.5 : 1.0;
  dc[p] = x1 ? 0.0 : wz * (0.5 * (rp + r[p + 1]));
  dc[n + p] = z1 ? 0.0 : wx * (0.5 * (rp + r[p + g.nx]));
  dc[2 * n + p] = (wz * (double)(x0 + x1) + wx * (double)(z0 + z1)) * sqrt(rp);
}

// out3 = {min m / sqrt(rho), max m / sqrt(rho), count of rho entries that are
// not finite and positive}: the slowness range the density-weighted equation
// propagates with (its local wavenumber is omega m / sqrt(rho)).
__global__ void __launch_bounds__(1024) k_check_density(size_t n, const double* __restrict__ m,
                                                        const double* __restrict__ rho, double* __restrict__ out3) {
  __shared__ double sh[3][16];
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = rho[i];
    if (!(isfinite(r) && r > 0.0)) {
      bad += 1.0;
    } else {
      const double v = m[i] / sqrt(r);
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    bad += __shfl_xor(bad, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wid] = lo;
    sh[1][wid] = hi;
    sh[2][wid] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      sh[0][0] = fmin(sh[0][0], sh[0][w]);
      sh[1][0] = fmax(sh[1][0], sh[1][w]);
      sh[2][0] += sh[2][w];
    }
    out3[0] = sh[0][0];
    out3[1] = sh[1][0];
    out3[2] = sh[2][0];
  }
}

// ---------------------------------------------------------------- 3D grids
// One node per thread on (nz, ny, nx) grids (hz_node3.h): neighbours are
// read from memory, the 2D tiling runs over the nz * ny rows.

__global__ void __launch_bounds__(kBlock) k_apply3(Grid g, Tiles t, int which, Batch bt,
                                                   const double2* __restrict__ x, double2* __restrict__ y,
                                                   size_t stride) {
  int slot, tile, iz, iy, ix;
  size_t p;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, g, iz, iy, ix, p)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double sre = which ? f.sM_re : f.sB_re, sim = which ? f.sM_im : f.sB_im;
  const NodeOp3 o = node_op3(iz, iy, ix, g, p, model_m(g, f)[p], f.omega, sre, sim);
  const double2* xs = x + (size_t)slot * stride;
  y[(size_t)slot * stride + p] = apply_op3(g, o, xs, p, iz, iy, ix, 1.0 / (g.h * g.h));
}

// u_out = u_in + w (b - M u_in) / diag(M); ZERO: u_in = 0 (as k_smooth)
template <bool ZERO>
__global__ void __launch_bounds__(kBlock) k_smooth3(Grid g, Tiles t, int lvl, double w_override, Batch bt,
                                                    const double2* __restrict__ b,
                                                    const double2* __restrict__ u_in,
                                                    double2* __restrict__ u_out, size_t stride, int coarse_only) {
  int slot, tile, iz, iy, ix;
  size_t p;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, g, iz, iy, ix, p)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  if (coarse_only && !f.coarse_jacobi) return;
  const double ih2 = 1.0 / (g.h * g.h);
  const NodeOp3 o = node_op3(iz, iy, ix, g, p, model_m(g, f)[p], f.omega, f.sM_re, f.sM_im);
  const double2 wdinv = w_override > 0.0 ? cscale(w_override, cinv(diag3(o.c, ih2))) : f.winv[lvl][p];
  const size_t base = (size_t)slot * stride;
  const double2 bp = b[base + p];
  double2 out;
  if (ZERO) {
    out = cmul(bp, wdinv);
  } else {
    const double2* us = u_in + base;
    const double2 res = csub(bp, apply_op3(g, o, us, p, iz, iy, ix, ih2));
    out = cadd(us[p], cmul(res, wdinv));
  }
  u_out[base + p] = out;
}

// One damped-Jacobi sweep on a 3D level from a given iterate with the
// level's tabulated w/D, marching along z: a wavefront owns kMarchW columns of
// one y-row (lane = column, from xs - 1; lanes 1 .. kMarchW store) and
// kMarchZ z-planes, two planes per step with all their loads issued
// together. z-neighbours stay in registers, x-neighbours come from the
// adjacent lanes. A block of kMarchWaves wavefronts owns that many
// neighbouring y-rows of one strip and z-chunk: every step each wavefront
// puts its row's iterate on the step's two planes in LDS (the planes it holds
// in registers anyway), the first and the last wavefront also the rows just
// below and above the block, and after one barrier every wavefront reads its
// y-neighbours there, so a row is read from memory once per block instead of
// by each of its neighbours. Rows past the grid are zero; their wavefronts
// load and store nothing and only take part in the barriers. The LDS rows
// are double-buffered by step parity: one barrier per step. Written in the
// Jacobi form (1 - w) u + (w/D)(b + (fz sz + fy sy + fx sx) / h^2), so the
// slowness is not read.
// FROM_ZERO: the two sweeps from u = 0 in one pass. The first gives
// u1 = (w/D) b, formed wherever the march reads u (u_in is not read), and the
// pass stores the second sweep from u1.
// PROLONG: the sweep starts from u_in + P e (e on the next coarser level gc,
// trilinear P), formed wherever the march reads the iterate: once per node,
// since the y-neighbour rows come through LDS (the block's edge wavefronts
// also form it on their halo rows), with each coarse plane interpolated to
// the row once and carried along the march. The prolongation then needs no
// pass of its own, and the corrected iterate is never stored.
// Shapes measured on the 129^3 benchmark box (step time): z-chunks of 4 to
// 32 planes, 1 to 16 wavefronts per block, with and without the LDS rows;
// 6 planes and 4 wavefronts sharing rows through LDS the fastest.
constexpr int kMarchW = 62;
constexpr int kMarchZ = 6;      // even: the march takes two planes per step
constexpr int kMarchWaves = 4;  // wavefronts (neighbouring y-rows) per block

template <bool FROM_ZERO, bool PROLONG>
__global__ void __launch_bounds__(64 * kMarchWaves) k_smooth3m(Grid g, int nstrip, int nchunk, int nyg, int groups,
                                                               int lvl, Batch bt, const double2* __restrict__ b,
                                                               const double2* __restrict__ u_in,
                                                               double2* __restrict__ u_out, size_t stride, Grid gc,
                                                               const double2* __restrict__ e, size_t sc) {
  static_assert(!(FROM_ZERO && PROLONG), "the prolongation corrects a given iterate");
  __shared__ double2 ysh[2][2][kMarchWaves + 2][64];  // [step parity][plane of the step][row slot][lane]
  int slot, grp;
  if (!decode_tile(bt, groups, slot, grp)) return;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int yg = grp % nyg, rest = grp / nyg;
  const int strip = rest % nstrip, chunk = rest / nstrip;
  const int iy0 = yg * kMarchWaves, iy = iy0 + wv;
  const bool row = iy < g.ny;          // the wavefront's row is in the grid
  const int iyc = min(iy, g.ny - 1);   // an address inside the grid for every wavefront
  const int lane = threadIdx.x % 64;
  const int x = strip * kMarchW - 1 + lane;
  const bool xin = x >= 0 && x < g.nx;
  const int xx = min(max(x, 0), g.nx - 1);
  const bool own = lane >= 1 && lane <= kMarchW && xin && row;
  const int z0 = chunk * kMarchZ, z1 = min(g.nz, z0 + kMarchZ);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double2* wd = f.winv[lvl];
  const double omw = 1.0 - f.wj[lvl];
  const double ih2 = 1.0 / (g.h * g.h);
  const size_t base = (size_t)slot * stride;
  const double2* us = FROM_ZERO ? nullptr : u_in + base;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const double wy = (iy == 0 || iy == g.ny - 1) ? 0.5 : 1.0, wx = (x == 0 || x == g.nx - 1) ? 0.5 : 1.0;
  const double2 zero = c2(0.0, 0.0);
  // the first wavefront also puts the row below the block in LDS (slot 0),
  // the last the row above it (slot kMarchWaves + 1); zero where that row is
  // outside the grid
  const bool edge = wv == 0 || wv == kMarchWaves - 1;
  const int hr = wv == 0 ? iy0 - 1 : iy0 + kMarchWaves;
  const bool halo = edge && hr >= 0 && hr < g.ny;
  const int hslot = wv == 0 ? 0 : kMarchWaves + 1;
  auto at_row = [&](int r, int z) { return (size_t)z * sz + (size_t)r * sy + xx; };
  auto at = [&](int z) { return at_row(iyc, z); };
  // the iterate the sweep starts from at node (z, r, xx) (PROLONG: without P e)
  auto uval = [&](int r, int z) {
    const size_t q = at_row(r, z);
    if constexpr (FROM_ZERO) return cmul(b[base + q], wd[q]);
    return us[q];
  };
  // the iterate on plane z of the wavefront's row, zero outside the grid
  auto plane = [&](int z) { return (row && z >= 0 && z < g.nz) ? keep(xin, uval(iyc, z)) : zero; };
  // the halo row's iterate on plane z (clamped into the grid: a second plane past it is not stored)
  auto hval = [&](int z) { return halo ? uval(hr, min(z, g.nz - 1)) : zero; };
  struct Row {
    double2 uc, ul, ur, bz, wdz;
  };
  auto centre = [&](int z, Row& r) {  // b and w/D at plane z of the row (clamped: a second plane past the grid)
    const size_t q = at(min(z, g.nz - 1));
    r.bz = row ? b[base + q] : zero;
    r.wdz = row ? wd[q] : zero;
  };
  auto step = [&](int z, const Row& r, double2 ua, double2 ub) {
    const double wz = (z == 0 || z == g.nz - 1) ? 0.5 : 1.0;
    const double fz = wy * wx, fy = wz * wx, fx = wz * wy;
    const double2 sxv = cadd(from_left(ub), from_right(ub));
    const double2 syv = cadd(r.ul, r.ur);
    const double2 szv = cadd(ua, r.uc);
    const double tx = ih2 * (fz * szv.x + fy * syv.x + fx * sxv.x) + r.bz.x;
    const double ty = ih2 * (fz * szv.y + fy * syv.y + fx * sxv.y) + r.bz.y;
    const double2 out =
        c2(omw * ub.x + (r.wdz.x * tx - r.wdz.y * ty), omw * ub.y + (r.wdz.x * ty + r.wdz.y * tx));
    if (own && z < z1) u_out[base + at(z)] = out;
  };
  // the step's exchange: this row's iterate on planes z (p0) and z + 1 (p1)
  // and the halo row's go to LDS; the y-neighbours come back
  auto exchange = [&](int z, double2 p0, double2 p1, double2 h0, double2 h1, Row& r0, Row& r1) {
    const int buf = ((z - z0) >> 1) & 1;
    ysh[buf][0][wv + 1][lane] = p0;
    ysh[buf][1][wv + 1][lane] = p1;
    if (edge) {
      ysh[buf][0][hslot][lane] = h0;
      ysh[buf][1][hslot][lane] = h1;
    }
    __syncthreads();
    r0.ul = ysh[buf][0][wv][lane];
    r0.ur = ysh[buf][0][wv + 2][lane];
    r1.ul = ysh[buf][1][wv][lane];
    r1.ur = ysh[buf][1][wv + 2][lane];
  };
  if constexpr (FROM_ZERO) {
    auto raw = [&](int z, double2& bq, double2& wq) {
      const bool in = row && z >= 0 && z < g.nz;
      const size_t q = at(in ? z : 0);
      bq = in ? b[base + q] : zero;
      wq = in ? wd[q] : zero;
    };
    double2 bq, wq;
    raw(z0 - 1, bq, wq);
    double2 ua = keep(xin, cmul(bq, wq));
    raw(z0, bq, wq);
    double2 ub = keep(xin, cmul(bq, wq));
    for (int z = z0; z < z1; z += 2) {
      Row r0, r1;
      r0.bz = bq;
      r0.wdz = wq;
      raw(z + 1, r1.bz, r1.wdz);
      raw(z + 2, bq, wq);
      r0.uc = keep(xin, cmul(r1.bz, r1.wdz));
      r1.uc = keep(xin, cmul(bq, wq));
      exchange(z, ub, r0.uc, hval(z), hval(z + 1), r0, r1);
      step(z, r0, ua, ub);
      step(z + 1, r1, ub, r0.uc);
      ua = r0.uc;
      ub = r1.uc;
    }
  } else if constexpr (PROLONG) {
    // P e on fine plane z: the coarse plane z/2 (z even) or the mean of the
    // coarse planes around it, each interpolated in y and x to the lane's
    // node (the order of interp3); a coarse plane serves two steps, so it is
    // formed once and carried
    const double2* es = e + (size_t)slot * sc;
    const int ox = xx & 1, Jx = xx >> 1, Jx1 = min(Jx + 1, gc.nx - 1);
    auto cline = [&](int Z, int Y) {
      const double2* r = es + ((size_t)Z * gc.ny + Y) * gc.nx;
      return ox ? cscale(0.5, cadd(r[Jx], r[Jx1])) : r[Jx];
    };
    auto cplane = [&](int r, int Z) {  // coarse plane Z (clamped into the grid) at the lane's node of row r
      Z = min(max(Z, 0), gc.nz - 1);
      const int Y = r >> 1, Y1 = min(Y + 1, gc.ny - 1);
      return (r & 1) ? cscale(0.5, cadd(cline(Z, Y), cline(Z, Y1))) : cline(Z, Y);
    };
    auto mean = [](double2 a, double2 c) { return cscale(0.5, cadd(a, c)); };
    // u + P e on plane z of the wavefront's row, zero outside the grid
    auto corrected = [&](int z, double2 pe) {
      return (row && z >= 0 && z < g.nz) ? keep(xin, cadd(us[at(z)], pe)) : zero;
    };
    // the halo row's u + P e on plane z (clamped into the grid: a second plane past it is not stored)
    auto hcorr = [&](int z, double2 pe) { return halo ? cadd(us[at_row(hr, min(z, g.nz - 1))], pe) : zero; };
    const int Z0 = z0 >> 1;  // z0 is even
    double2 cp = row ? cplane(iyc, Z0 - 1) : zero, cc = row ? cplane(iyc, Z0) : zero;
    double2 hc = halo ? cplane(hr, Z0) : zero;
    double2 ua = corrected(z0 - 1, mean(cp, cc)), ub = corrected(z0, cc);
    for (int z = z0; z < z1; z += 2) {
      const int Z = z >> 1;
      const double2 cn = row ? cplane(iyc, Z + 1) : zero, hn = halo ? cplane(hr, Z + 1) : zero;
      Row r0, r1;
      r0.uc = corrected(z + 1, mean(cc, cn));
      r1.uc = corrected(z + 2, cn);
      centre(z, r0);
      centre(z + 1, r1);
      exchange(z, ub, r0.uc, hcorr(z, hc), hcorr(z + 1, mean(hc, hn)), r0, r1);
      step(z, r0, ua, ub);
      step(z + 1, r1, ub, r0.uc);
      ua = r0.uc;
      ub = r1.uc;
      cc = cn;
      hc = hn;
    }
  } else {
    double2 ua = plane(z0 - 1), ub = plane(z0);
    for (int z = z0; z < z1; z += 2) {
      Row r0, r1;
      r0.uc = plane(z + 1);
      r1.uc = plane(z + 2);
      centre(z, r0);
      centre(z + 1, r1);
      exchange(z, ub, r0.uc, hval(z), hval(z + 1), r0, r1);
      step(z, r0, ua, ub);
      step(z + 1, r1, ub, r0.uc);
      ua = r0.uc;
      ub = r1.uc;
    }
  }
}

// Prolongation and both post-sweeps of a 3D level in one march (nu2 >= 2,
// constant density): u1 = sweep(u + P e) as k_smooth3m<false, true> forms
// it, and u2 = sweep(u1) one plane behind; neither u + P e nor u1 is stored.
// The second sweep needs the first on a ring of nodes around what it stores,
// so the blocks overlap: a block of kPostWaves wavefronts runs the first
// sweep on kPostWaves neighbouring y-rows and the second on the inner
// kPostWaves - 2 of them; a wavefront owns kPostW + 4 columns, the first
// sweep is right on all but its outer lanes and the second is stored on the
// inner kPostW; a chunk of planes starts one step (two planes) early. The
// first sweep's y-neighbours come through one LDS exchange per step (the
// edge wavefronts also put the rows just outside the block there), the
// second's through another; with two barriers per step one buffer of each
// suffices. The arithmetic is k_smooth3m's.
// Measured on the 129^3 benchmark box (step time): 8 wavefronts and 12 planes
// 460 ms (16 planes 462, 8 planes 474; 6 or 16 wavefronts at 8 planes 550 and
// 473), against 472 ms for the two sweeps as separate marches.
constexpr int kPostW = 60;
constexpr int kPostZ = 12;     // planes per chunk (even)
constexpr int kPostWaves = 8;  // wavefronts (y-rows of the first sweep) per block

__global__ void __launch_bounds__(64 * kPostWaves) k_post3m(Grid g, Grid gc, int nstrip, int nchunk, int nyg,
                                                            int groups, int lvl, Batch bt,
                                                            const double2* __restrict__ b,
                                                            const double2* __restrict__ u_in,
                                                            const double2* __restrict__ e,
                                                            double2* __restrict__ u_out, size_t stride, size_t sc) {
  __shared__ double2 ysh0[2][kPostWaves + 2][64];  // u + P e: [plane of the step][row slot][lane]
  __shared__ double2 ysh1[2][kPostWaves][64];      // the first sweep
  int slot, grp;
  if (!decode_tile(bt, groups, slot, grp)) return;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int yg = grp % nyg, rest = grp / nyg;
  const int strip = rest % nstrip, chunk = rest / nstrip;
  const int iy = yg * (kPostWaves - 2) - 1 + wv;  // this wavefront's row; the block stores rows of waves 1 .. W - 2
  const bool row = iy >= 0 && iy < g.ny;
  const int iyc = min(max(iy, 0), g.ny - 1);       // an address inside the grid for every wavefront
  const bool inner = wv >= 1 && wv <= kPostWaves - 2;
  const int lane = threadIdx.x % 64;
  const int x = strip * kPostW - 2 + lane;
  const bool xin = x >= 0 && x < g.nx;
  const int xx = min(max(x, 0), g.nx - 1);
  const bool own = lane >= 2 && lane <= kPostW + 1 && xin && row && inner;
  const int z0 = chunk * kPostZ, z1 = min(g.nz, z0 + kPostZ);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double2* wd = f.winv[lvl];
  const double omw = 1.0 - f.wj[lvl];
  const double ih2 = 1.0 / (g.h * g.h);
  const size_t base = (size_t)slot * stride;
  const double2* us = u_in + base;
  const double2* es = e + (size_t)slot * sc;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const double wy = (iy == 0 || iy == g.ny - 1) ? 0.5 : 1.0, wx = (x == 0 || x == g.nx - 1) ? 0.5 : 1.0;
  const double2 zero = c2(0.0, 0.0);
  const bool edge = wv == 0 || wv == kPostWaves - 1;
  const int hr = wv == 0 ? iy - 1 : iy + 1;
  const bool halo = edge && hr >= 0 && hr < g.ny;
  const int hslot = wv == 0 ? 0 : kPostWaves + 1;
  auto at_row = [&](int r, int z) { return (size_t)z * sz + (size_t)r * sy + xx; };
  auto inz = [&](int z) { return z >= 0 && z < g.nz; };
  auto clz = [&](int z) { return min(max(z, 0), g.nz - 1); };
  // P e (as k_smooth3m<false, true>: coarse planes interpolated to the row and carried)
  const int ox = xx & 1, Jx = xx >> 1, Jx1 = min(Jx + 1, gc.nx - 1);
  auto cline = [&](int Z, int Y) {
    const double2* r = es + ((size_t)Z * gc.ny + Y) * gc.nx;
    return ox ? cscale(0.5, cadd(r[Jx], r[Jx1])) : r[Jx];
  };
  auto cplane = [&](int r, int Z) {
    Z = min(max(Z, 0), gc.nz - 1);
    const int Y = r >> 1, Y1 = min(Y + 1, gc.ny - 1);
    return (r & 1) ? cscale(0.5, cadd(cline(Z, Y), cline(Z, Y1))) : cline(Z, Y);
  };
  auto mean = [](double2 a, double2 c) { return cscale(0.5, cadd(a, c)); };
  auto corrected = [&](int z, double2 pe) {
    return (row && inz(z)) ? keep(xin, cadd(us[at_row(iyc, z)], pe)) : zero;
  };
  auto hcorr = [&](int z, double2 pe) { return halo ? cadd(us[at_row(hr, clz(z))], pe) : zero; };
  // one sweep at plane z of the row from (ua, ub, uc) on planes z - 1, z, z + 1 and the y-neighbours
  auto jac = [&](int z, double2 ua, double2 ub, double2 uc, double2 ul, double2 ur, double2 bz, double2 wdz) {
    const double wz = (z == 0 || z == g.nz - 1) ? 0.5 : 1.0;
    const double fz = wy * wx, fy = wz * wx, fx = wz * wy;
    const double2 sxv = cadd(from_left(ub), from_right(ub));
    const double2 syv = cadd(ul, ur);
    const double2 szv = cadd(ua, uc);
    const double tx = ih2 * (fz * szv.x + fy * syv.x + fx * sxv.x) + bz.x;
    const double ty = ih2 * (fz * szv.y + fy * syv.y + fx * sxv.y) + bz.y;
    return c2(omw * ub.x + (wdz.x * tx - wdz.y * ty), omw * ub.y + (wdz.x * ty + wdz.y * tx));
  };
  auto centre = [&](int z, double2& bz, double2& wdz) {
    const bool in = row && inz(z);
    const size_t q = at_row(iyc, clz(z));
    bz = in ? b[base + q] : zero;
    wdz = in ? wd[q] : zero;
  };
  const int zs = z0 - 2;  // the march starts a step early
  const int Zs = zs >> 1;
  double2 cc = row ? cplane(iyc, Zs) : zero, hc = halo ? cplane(hr, Zs) : zero;
  double2 ua = corrected(zs - 1, mean(row ? cplane(iyc, Zs - 1) : zero, cc)), ub = corrected(zs, cc);
  double2 v1a = zero, v1b = zero;  // the first sweep on planes z - 2, z - 1
  double2 bp = zero, wp = zero;    // b and w/D on plane z - 1
  for (int z = zs; z <= z1; z += 2) {
    const int Z = z >> 1;
    const double2 cn = row ? cplane(iyc, Z + 1) : zero, hn = halo ? cplane(hr, Z + 1) : zero;
    const double2 u0c1 = corrected(z + 1, mean(cc, cn)), u0c2 = corrected(z + 2, cn);
    double2 b0, w0, b1, w1;
    centre(z, b0, w0);
    centre(z + 1, b1, w1);
    // the first sweep on planes z and z + 1
    ysh0[0][wv + 1][lane] = ub;
    ysh0[1][wv + 1][lane] = u0c1;
    if (edge) {
      ysh0[0][hslot][lane] = hcorr(z, hc);
      ysh0[1][hslot][lane] = hcorr(z + 1, mean(hc, hn));
    }
    __syncthreads();
    double2 u1z = jac(z, ua, ub, u0c1, ysh0[0][wv][lane], ysh0[0][wv + 2][lane], b0, w0);
    double2 u1z1 = jac(z + 1, ub, u0c1, u0c2, ysh0[1][wv][lane], ysh0[1][wv + 2][lane], b1, w1);
    u1z = (row && inz(z)) ? keep(xin, u1z) : zero;
    u1z1 = (row && inz(z + 1)) ? keep(xin, u1z1) : zero;
    // the second on planes z - 1 and z
    ysh1[0][wv][lane] = v1b;
    ysh1[1][wv][lane] = u1z;
    __syncthreads();
    if (inner) {
      const double2 o0 = jac(z - 1, v1a, v1b, u1z, ysh1[0][wv - 1][lane], ysh1[0][wv + 1][lane], bp, wp);
      const double2 o1 = jac(z, v1b, u1z, u1z1, ysh1[1][wv - 1][lane], ysh1[1][wv + 1][lane], b0, w0);
      if (own && z - 1 >= z0 && z - 1 < z1) u_out[base + at_row(iyc, z - 1)] = o0;
      if (own && z >= z0 && z < z1) u_out[base + at_row(iyc, z)] = o1;
    }
    ua = u0c1;
    ub = u0c2;
    v1a = u1z;
    v1b = u1z1;
    bp = b1;
    wp = w1;
    cc = cn;
    hc = hn;
  }
}

__global__ void k_winv3(Grid g, double omega, double s_re, double s_im, double w, double2* __restrict__ winv) {
  const size_t n = (size_t)g.nz * g.ny * g.nx;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int ix = (int)(p % g.nx);
  const int r = (int)(p / g.nx);
  const int iz = r / g.ny, iy = r - iz * g.ny;
  const NodeOp3 o = node_op3(iz, iy, ix, g, p, g.m[p], omega, s_re, s_im);
  winv[p] = cscale(w, cinv(diag3(o.c, 1.0 / (g.h * g.h))));
}

// weight of fine offset d in {-1, 0, 1} around coarse node J in P^T (see k_restrict)
__device__ __forceinline__ double pt_weight(int d, int J, int nf) {
  return (d == 0 || (d == 1 && 2 * J + 2 == nf)) ? 1.0 : 0.5;
}

// bc = 2^-3 P^T (b - M u), one thread per coarse node, the residual formed
// at each of the (up to) 27 fine nodes it gathers
__global__ void __launch_bounds__(kBlock) k_restrict3(Grid gf, Grid gc, Tiles t, Batch bt,
                                                      const double2* __restrict__ b,
                                                      const double2* __restrict__ u,
                                                      double2* __restrict__ bc, size_t sf, size_t sc) {
  int slot, tile, Iz, Iy, Ix;
  size_t P;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, gc, Iz, Iy, Ix, P)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double ih2 = 1.0 / (gf.h * gf.h);
  const double2* bs = b + (size_t)slot * sf;
  const double2* us = u + (size_t)slot * sf;
  double2 acc = c2(0.0, 0.0);
  for (int dz = -1; dz <= 1; ++dz) {
    const int iz = 2 * Iz + dz;
    if (iz < 0 || iz >= gf.nz) continue;
    const double wz = pt_weight(dz, Iz, gf.nz);
    for (int dy = -1; dy <= 1; ++dy) {
      const int iy = 2 * Iy + dy;
      if (iy < 0 || iy >= gf.ny) continue;
      const double wzy = wz * pt_weight(dy, Iy, gf.ny);
      for (int dx = -1; dx <= 1; ++dx) {
        const int ix = 2 * Ix + dx;
        if (ix < 0 || ix >= gf.nx) continue;
        const size_t p = ((size_t)iz * gf.ny + iy) * gf.nx + ix;
        const NodeOp3 o = node_op3(iz, iy, ix, gf, p, model_m(gf, f)[p], f.omega, f.sM_re, f.sM_im);
        const double2 r = csub(bs[p], apply_op3(gf, o, us, p, iz, iy, ix, ih2));
        acc = cadd(acc, cscale(wzy * pt_weight(dx, Ix, gf.nx), r));
      }
    }
  }
  bc[(size_t)slot * sc + P] = cscale(0.125, acc);
}

// r = b - M u on a 3D level, for the restriction below
__global__ void __launch_bounds__(kBlock) k_residual3(Grid g, Tiles t, Batch bt, const double2* __restrict__ b,
                                                      const double2* __restrict__ u, double2* __restrict__ r,
                                                      size_t stride) {
  int slot, tile, iz, iy, ix;
  size_t p;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, g, iz, iy, ix, p)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  const NodeOp3 o = node_op3(iz, iy, ix, g, p, model_m(g, f)[p], f.omega, f.sM_re, f.sM_im);
  r[base + p] = csub(b[base + p], apply_op3(g, o, u + base, p, iz, iy, ix, 1.0 / (g.h * g.h)));
}

// bc = 2^-3 P^T r from a stored fine residual (the weights of k_restrict3)
__global__ void __launch_bounds__(kBlock) k_restrict_r3(Grid gf, Grid gc, Tiles t, Batch bt,
                                                        const double2* __restrict__ r, double2* __restrict__ bc,
                                                        size_t sf, size_t sc) {
  int slot, tile, Iz, Iy, Ix;
  size_t P;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, gc, Iz, Iy, Ix, P)) return;
  const double2* rs = r + (size_t)slot * sf;
  // offsets past the grid read the centre fine node (2I, always inside) with weight zero, so
  // the 27 loads carry no branches and are all issued before the sum
  int zi[3], yi[3], xi[3];
  double wz[3], wy[3], wx[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int iz = 2 * Iz + d - 1, iy = 2 * Iy + d - 1, ix = 2 * Ix + d - 1;
    const bool inz = iz >= 0 && iz < gf.nz, iny = iy >= 0 && iy < gf.ny, inx = ix >= 0 && ix < gf.nx;
    zi[d] = inz ? iz : 2 * Iz;
    yi[d] = iny ? iy : 2 * Iy;
    xi[d] = inx ? ix : 2 * Ix;
    wz[d] = inz ? pt_weight(d - 1, Iz, gf.nz) : 0.0;
    wy[d] = iny ? pt_weight(d - 1, Iy, gf.ny) : 0.0;
    wx[d] = inx ? pt_weight(d - 1, Ix, gf.nx) : 0.0;
  }
  double2 v[27];
#pragma unroll
  for (int k = 0; k < 27; ++k)
    v[k] = rs[((size_t)zi[k / 9] * gf.ny + yi[(k / 3) % 3]) * gf.nx + xi[k % 3]];
  double2 acc = c2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 27; ++k) acc = cadd(acc, cscale(wz[k / 9] * wy[(k / 3) % 3] * wx[k % 3], v[k]));
  bc[(size_t)slot * sc + P] = cscale(0.125, acc);
}

// u_out = u_in + P e (u_out may be u_in)
__global__ void __launch_bounds__(kBlock) k_prolong3(Grid gf, Grid gc, Tiles t, Batch bt,
                                                     const double2* __restrict__ e, const double2* u_in,
                                                     double2* u_out, size_t sf, size_t sc) {
  int slot, tile, iz, iy, ix;
  size_t p;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, gf, iz, iy, ix, p)) return;
  const size_t q = (size_t)slot * sf + p;
  u_out[q] = cadd(u_in[q], interp3(e + (size_t)slot * sc, iz, iy, ix, gc.nz, gc.ny, gc.nx));
}

// Prolongation, correction and one damped-Jacobi sweep in one pass (as
// k_prolong_smooth): u3 = u2 + P e at the node and its six neighbours.
__global__ void __launch_bounds__(kBlock) k_prolong_smooth3(Grid gf, Grid gc, Tiles t, int lvl, Batch bt,
                                                            const double2* __restrict__ e,
                                                            const double2* __restrict__ b,
                                                            const double2* __restrict__ u2,
                                                            double2* __restrict__ u_out, size_t sf, size_t sc) {
  int slot, tile, iz, iy, ix;
  size_t p;
  if (!decode_tile(bt, t.per_slot, slot, tile) || !node3_of(t, tile, gf, iz, iy, ix, p)) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double ih2 = 1.0 / (gf.h * gf.h);
  const size_t base = (size_t)slot * sf;
  const double2* es = e + (size_t)slot * sc;
  const double2* us = u2 + base;
  auto u3_at = [&](int qz, int qy, int qx) -> double2 {
    return cadd(us[((size_t)qz * gf.ny + qy) * gf.nx + qx], interp3(es, qz, qy, qx, gc.nz, gc.ny, gc.nx));
  };
  const NodeOp3 o = node_op3(iz, iy, ix, gf, p, model_m(gf, f)[p], f.omega, f.sM_re, f.sM_im);
  const double2 u3p = u3_at(iz, iy, ix);
  const double2 res = csub(b[base + p], apply_op3_at(gf, o, iz, iy, ix, ih2, u3p, [&](int dz, int dy, int dx) {
                             return u3_at(iz + dz, iy + dy, ix + dx);
                           }));
  u_out[base + p] = cadd(u3p, cmul(res, f.winv[lvl][p]));
}

// Dense M on the coarsest 3D grid for every frequency: A[f][i][j].
__global__ void k_assemble_dense3(Grid g, int nfreq, const FreqTab* __restrict__ ft, double2* __restrict__ A) {
  const size_t nc = (size_t)g.nz * g.ny * g.nx;
  const size_t total = nc * nc * nfreq;
  const double ih2 = 1.0 / (g.h * g.h);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int f = (int)(e / (nc * nc));
    const size_t rem = e - (size_t)f * nc * nc;
    const int i = (int)(rem / nc), j = (int)(rem - (size_t)i * nc);
    const int ix = i % g.nx, iy = (i / g.nx) % g.ny, iz = i / (g.nx * g.ny);
    const int jx = j % g.nx, jy = (j / g.nx) % g.ny, jz = j / (g.nx * g.ny);
    const NodeOp3 o = node_op3(iz, iy, ix, g, i, model_m(g, ft[f])[i], ft[f].omega, ft[f].sM_re, ft[f].sM_im);
    const NodeC3& c = o.c;
    double2 val = c2(0.0, 0.0);
    if (i == j) {
      val = diag3(c, ih2);
    } else if (jz == iz && jy == iy && (jx == ix - 1 || jx == ix + 1)) {
      val = c2(-(g.rho ? o.cq[jx == ix - 1 ? 0 : 1] : c.fx) * ih2, 0.0);
    } else if (jz == iz && jx == ix && (jy == iy - 1 || jy == iy + 1)) {
      val = c2(-(g.rho ? o.cq[jy == iy - 1 ? 2 : 3] : c.fy) * ih2, 0.0);
    } else if (jy == iy && jx == ix && (jz == iz - 1 || jz == iz + 1)) {
      val = c2(-(g.rho ? o.cq[jz == iz - 1 ? 4 : 5] : c.fz) * ih2, 0.0);
    }
    A[e] = val;
  }
}

__global__ void k_inject3(Grid gf, double* __restrict__ mc) {
  const int ncx = (gf.nx + 1) / 2, ncy = (gf.ny + 1) / 2, ncz = (gf.nz + 1) / 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncx * ncy * ncz) return;
  const int Ix = i % ncx, Iy = (i / ncx) % ncy, Iz = i / (ncx * ncy);
  mc[i] = gf.m[((size_t)2 * Iz * gf.ny + 2 * Iy) * gf.nx + 2 * Ix];
}

// ---------------------------------------------------------------- launchers
static inline dim3 grid1(long long blocks) { return dim3((unsigned)blocks); }

// the row tiling of a 3D grid
static inline Tiles tiles3(const Grid& g) { return grid_tiles(g.nz * g.ny, g.nx, 3); }

hipError_t launch_apply(int dim, const Grid& g, int lvl, int which, const Batch& bt, int cap,
                        const double2* x, double2* y, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (dim == 3) {
    const Tiles t = tiles3(g);
    hipLaunchKernelGGL(k_apply3, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, g, t, which, bt, x, y, stride);
    return hipGetLastError();
  }
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (dim == 2)
    hipLaunchKernelGGL(k_apply<true>, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, g, t, lvl, which, bt, x, y, stride);
  else
    hipLaunchKernelGGL(k_apply<false>, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, g, t, lvl, which, bt, x, y, stride);
  return hipGetLastError();
}

// the marching 3D sweep (from u_in, or both sweeps from zero)
hipError_t launch_march3(const Grid& g, int lvl, const Batch& bt, int cap, bool from_zero, const double2* b,
                         const double2* u_in, double2* u_out, size_t stride, hipStream_t st, const Grid* gc,
                         const double2* e, size_t sc) {
  if (cap <= 0) return hipSuccess;
  if (g.rho) return hipErrorInvalidValue;  // constant density only
  if (e && (!gc || from_zero || !u_in || gc->nz != coarse_n(g.nz) || gc->ny != coarse_n(g.ny) ||
            gc->nx != coarse_n(g.nx)))
    return hipErrorInvalidValue;
  const int nstrip = (g.nx + kMarchW - 1) / kMarchW, nchunk = (g.nz + kMarchZ - 1) / kMarchZ;
  const int nyg = (g.ny + kMarchWaves - 1) / kMarchWaves;
  const int groups = nyg * nstrip * nchunk;
  const dim3 gr = grid1(tile_blocks(groups, cap)), bl(64 * kMarchWaves);
  const Grid gcc = e ? *gc : g;
  if (from_zero)
    hipLaunchKernelGGL((k_smooth3m<true, false>), gr, bl, 0, st, g, nstrip, nchunk, nyg, groups, lvl, bt, b, u_in,
                       u_out, stride, gcc, nullptr, (size_t)0);
  else if (e)
    hipLaunchKernelGGL((k_smooth3m<false, true>), gr, bl, 0, st, g, nstrip, nchunk, nyg, groups, lvl, bt, b, u_in,
                       u_out, stride, gcc, e, sc);
  else
    hipLaunchKernelGGL((k_smooth3m<false, false>), gr, bl, 0, st, g, nstrip, nchunk, nyg, groups, lvl, bt, b, u_in,
                       u_out, stride, gcc, nullptr, (size_t)0);
  return hipGetLastError();
}

hipError_t launch_post3(const Grid& g, const Grid& gc, int lvl, const Batch& bt, int cap, const double2* b,
                        const double2* u_in, const double2* e, double2* u_out, size_t stride, size_t sc,
                        hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (g.rho || !u_in || !e || u_in == u_out) return hipErrorInvalidValue;  // constant density; u_out apart
  if (gc.nz != coarse_n(g.nz) || gc.ny != coarse_n(g.ny) || gc.nx != coarse_n(g.nx)) return hipErrorInvalidValue;
  const int nstrip = (g.nx + kPostW - 1) / kPostW, nchunk = (g.nz + kPostZ - 1) / kPostZ;
  const int nyg = (g.ny + kPostWaves - 3) / (kPostWaves - 2);
  const int groups = nyg * nstrip * nchunk;
  hipLaunchKernelGGL(k_post3m, grid1(tile_blocks(groups, cap)), dim3(64 * kPostWaves), 0, st, g, gc, nstrip, nchunk,
                     nyg, groups, lvl, bt, b, u_in, e, u_out, stride, sc);
  return hipGetLastError();
}

hipError_t launch_smooth(int dim, const Grid& g, int lvl, double w_override, const Batch& bt,
                         int cap, const double2* b, const double2* u_in, double2* u_out,
                         size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  // (the marching sweep has constant density only)
  if (dim == 3 && u_in && w_override <= 0.0 && !g.rho)
    return launch_march3(g, lvl, bt, cap, false, b, u_in, u_out, stride, st);
  if (dim == 3) {
    const Tiles t = tiles3(g);
    const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
    if (u_in)
      hipLaunchKernelGGL(k_smooth3<false>, gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride, 0);
    else
      hipLaunchKernelGGL(k_smooth3<true>, gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride, 0);
    return hipGetLastError();
  }
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  // the LDS-tiled form has constant density only
  if (dim == 2 && u_in && w_override <= 0.0 && !g.rho) {
    const int ntx = (g.nx + kTX - 1) / kTX, ntz = (g.nz + kTZ - 1) / kTZ;
    hipLaunchKernelGGL(k_smooth_t, grid1(tile_blocks(ntx * ntz, cap)), dim3(kBlock), 0, st, g, ntx, ntx * ntz, lvl,
                       bt, b, u_in, u_out, stride);
    return hipGetLastError();
  }
  if (dim == 2) {
    if (u_in)
      hipLaunchKernelGGL((k_smooth<true, false>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride, 0);
    else
      hipLaunchKernelGGL((k_smooth<true, true>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride, 0);
  } else {
    if (u_in)
      hipLaunchKernelGGL((k_smooth<false, false>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride, 0);
    else
      hipLaunchKernelGGL((k_smooth<false, true>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride, 0);
  }
  return hipGetLastError();
}

hipError_t launch_restrict(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                           const double2* b, const double2* u, double2* bc, size_t sf, size_t sc,
                           hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (dim == 3) {
    const Tiles t = tiles3(gc);
    hipLaunchKernelGGL(k_restrict3, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, gf, gc, t, bt, b, u,
                       bc, sf, sc);
    return hipGetLastError();
  }
  const Tiles t = grid_tiles(gc.nz, gc.nx, dim);
  if (dim == 2 && !gf.rho) {
    const int ntx = (gc.nx + kRtx - 1) / kRtx, ntz = (gc.nz + kRtz - 1) / kRtz;
    hipLaunchKernelGGL(k_restrict_tiled, grid1(tile_blocks(ntx * ntz, cap)), dim3(kRtx * kRtz), 0, st, gf, gc,
                       ntx, ntx * ntz, bt, b, u, bc, sf, sc);
  } else if (dim == 2) {
    hipLaunchKernelGGL(k_restrict<true>, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, gf, gc, t, bt,
                       b, u, bc, sf, sc);
  } else {
    hipLaunchKernelGGL(k_restrict<false>, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, gf, gc, t, bt,
                       b, u, bc, sf, sc);
  }
  return hipGetLastError();
}

hipError_t launch_restrict_via(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                               const double2* b, const double2* u, double2* scratch, double2* bc, size_t sf,
                               size_t sc, hipStream_t st) {
  if (dim != 3) return launch_restrict(dim, gf, gc, bt, cap, b, u, bc, sf, sc, st);
  if (cap <= 0) return hipSuccess;
  const Tiles tf = tiles3(gf), tc = tiles3(gc);
  hipLaunchKernelGGL(k_residual3, grid1(tile_blocks(tf.per_slot, cap)), dim3(kBlock), 0, st, gf, tf, bt, b, u,
                     scratch, sf);
  hipLaunchKernelGGL(k_restrict_r3, grid1(tile_blocks(tc.per_slot, cap)), dim3(kBlock), 0, st, gf, gc, tc, bt,
                     scratch, bc, sf, sc);
  return hipGetLastError();
}

hipError_t launch_prolong(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                          const double2* e, const double2* u_in, double2* u_out, size_t sf,
                          size_t sc, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (dim == 3) {
    const Tiles t = tiles3(gf);
    hipLaunchKernelGGL(k_prolong3, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, gf, gc, t, bt, e, u_in,
                       u_out, sf, sc);
    return hipGetLastError();
  }
  const Tiles t = grid_tiles(gf.nz, gf.nx, dim);
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  if (dim == 2)
    hipLaunchKernelGGL(k_prolong<true>, gr, dim3(kBlock), 0, st, gf, gc, t, bt, e, u_in, u_out, sf, sc);
  else
    hipLaunchKernelGGL(k_prolong<false>, gr, dim3(kBlock), 0, st, gf, gc, t, bt, e, u_in, u_out, sf, sc);
  return hipGetLastError();
}

hipError_t launch_pre2(int dim, const Grid& g, int lvl, int mode, const Batch& bt, int cap,
                       const double2* in_a, const double2* in_b, const double2* in_c, double2* bout,
                       double2* u2, size_t stride, hipStream_t st) {
  // 2D grids take the fused pre-smoothing and restriction kernel (launch_pre2r);
  // constant density only
  if (dim != 1 || g.rho) return hipErrorInvalidValue;
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  const RhsIn in{in_a, in_b, in_c};
#define HZ_PRE2(M) hipLaunchKernelGGL((k_pre2<false, M>), gr, dim3(kBlock), 0, st, g, t, lvl, bt, in, bout, u2, stride)
  if (mode == 0) HZ_PRE2(0);
  else if (mode == 1) HZ_PRE2(1);
  else HZ_PRE2(2);
#undef HZ_PRE2
  return hipGetLastError();
}

hipError_t launch_prolong_smooth(int dim, const Grid& gf, const Grid& gc, int lvl, const Batch& bt,
                                 int cap, const double2* e, const double2* b, const double2* u2,
                                 double2* u_out, size_t sf, size_t sc, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (dim == 3) {
    const Tiles t = tiles3(gf);
    hipLaunchKernelGGL(k_prolong_smooth3, grid1(tile_blocks(t.per_slot, cap)), dim3(kBlock), 0, st, gf, gc, t, lvl,
                       bt, e, b, u2, u_out, sf, sc);
    return hipGetLastError();
  }
  const Tiles t = grid_tiles(gf.nz, gf.nx, dim);
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  if (dim == 2 && !gf.rho) {
    const int ntx = (gf.nx + kTX - 1) / kTX, ntz = (gf.nz + kTZ - 1) / kTZ;
    hipLaunchKernelGGL(k_prolong_smooth_t, grid1(tile_blocks(ntx * ntz, cap)), dim3(kBlock), 0, st, gf, gc, ntx,
                       ntx * ntz, lvl, bt, e, b, u2, u_out, sf, sc);
  } else if (dim == 2)
    hipLaunchKernelGGL(k_prolong_smooth<true>, gr, dim3(kBlock), 0, st, gf, gc, t, lvl, bt, e, b, u2, u_out, sf, sc);
  else
    hipLaunchKernelGGL(k_prolong_smooth<false>, gr, dim3(kBlock), 0, st, gf, gc, t, lvl, bt, e, b, u2, u_out, sf, sc);
  return hipGetLastError();
}

hipError_t launch_coarse_jacobi(int dim, const Grid& g, int lvl, double w, int sweeps, const Batch& bt, int cap,
                                const double2* b, double2* tmp, double2* u_out, size_t stride, hipStream_t st) {
  if (cap <= 0 || sweeps < 1) return hipSuccess;
  const Tiles t = dim == 3 ? tiles3(g) : grid_tiles(g.nz, g.nx, dim);
  const dim3 gr = grid1(tile_blocks(t.per_slot, cap));
  // ping-pong so that the last sweep lands in u_out
  double2* cur = (sweeps % 2 == 1) ? u_out : tmp;
  if (dim == 3)
    hipLaunchKernelGGL(k_smooth3<true>, gr, dim3(kBlock), 0, st, g, t, lvl, w, bt, b, nullptr, cur, stride, 1);
  else if (dim == 2)
    hipLaunchKernelGGL((k_smooth<true, true>), gr, dim3(kBlock), 0, st, g, t, lvl, w, bt, b, nullptr, cur, stride, 1);
  else
    hipLaunchKernelGGL((k_smooth<false, true>), gr, dim3(kBlock), 0, st, g, t, lvl, w, bt, b, nullptr, cur, stride, 1);
  for (int k = 1; k < sweeps; ++k) {
    double2* nxt = (cur == u_out) ? tmp : u_out;
    if (dim == 3)
      hipLaunchKernelGGL(k_smooth3<false>, gr, dim3(kBlock), 0, st, g, t, lvl, w, bt, b, cur, nxt, stride, 1);
    else if (dim == 2)
      hipLaunchKernelGGL((k_smooth<true, false>), gr, dim3(kBlock), 0, st, g, t, lvl, w, bt, b, cur, nxt, stride, 1);
    else
      hipLaunchKernelGGL((k_smooth<false, false>), gr, dim3(kBlock), 0, st, g, t, lvl, w, bt, b, cur, nxt, stride, 1);
    cur = nxt;
  }
  return hipGetLastError();
}

hipError_t launch_coarse_solve(int nc, int nfreq, int nrhs, const Batch& bt, const double2* bc,
                               double2* uc, size_t stride, hipStream_t st) {
  const int row_tiles = (nc + 15) / 16;
  const dim3 gr((row_tiles + kCoarseWaves - 1) / kCoarseWaves, (nrhs + 15) / 16, nfreq);
  hipLaunchKernelGGL(k_coarse, gr, dim3(kCoarseWaves * 64), 0, st, nc, bt, bc, uc, stride);
  return hipGetLastError();
}

hipError_t launch_pcr(const Grid& g, const Batch& bt, int cap, const double2* b, double2* u,
                      size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (g.nx > kPcrMax) return hipErrorInvalidValue;
  const size_t lds = (size_t)4 * g.nx * sizeof(double2);
  hipLaunchKernelGGL(k_pcr, dim3(cap), dim3(1024), lds, st, g, bt, b, u, stride);
  return hipGetLastError();
}

static inline unsigned flat_blocks(size_t total) {
  size_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return (unsigned)b;
}

hipError_t launch_winv(int dim, const Grid& g, double omega, double s_re, double s_im, double w,
                       double2* winv, hipStream_t st) {
  const size_t n = (size_t)g.nz * g.ny * g.nx;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dim == 3)
    hipLaunchKernelGGL(k_winv3, dim3(nb), dim3(256), 0, st, g, omega, s_re, s_im, w, winv);
  else if (dim == 2)
    hipLaunchKernelGGL(k_winv<true>, dim3(nb), dim3(256), 0, st, g, omega, s_re, s_im, w, winv);
  else
    hipLaunchKernelGGL(k_winv<false>, dim3(nb), dim3(256), 0, st, g, omega, s_re, s_im, w, winv);
  return hipGetLastError();
}

hipError_t launch_assemble_dense(int dim, const Grid& g, int nfreq, const FreqTab* ft, double2* A,
                                 hipStream_t st) {
  const size_t nc = (size_t)g.nz * g.ny * g.nx;
  const unsigned nb = flat_blocks(nc * nc * nfreq);
  if (dim == 3)
    hipLaunchKernelGGL(k_assemble_dense3, dim3(nb), dim3(256), 0, st, g, nfreq, ft, A);
  else if (dim == 2)
    hipLaunchKernelGGL(k_assemble_dense<true>, dim3(nb), dim3(256), 0, st, g, nfreq, ft, A);
  else
    hipLaunchKernelGGL(k_assemble_dense<false>, dim3(nb), dim3(256), 0, st, g, nfreq, ft, A);
  return hipGetLastError();
}

hipError_t launch_gj_step(int nc, int nfreq, int k, const double2* A_in, double2* A_out,
                          hipStream_t st) {
  const unsigned nb = flat_blocks((size_t)nc * nc * nfreq);
  hipLaunchKernelGGL(k_gj_step, dim3(nb), dim3(256), 0, st, nc, nfreq, k, A_in, A_out);
  return hipGetLastError();
}

hipError_t launch_point_rhs(size_t n, int nsrc, const int* nodes, const double2* amp, double scale,
                            double2* b, hipStream_t st) {
  hipLaunchKernelGGL(k_point_rhs_zero, dim3(flat_blocks(n * nsrc)), dim3(256), 0, st, n * nsrc, b);
  hipLaunchKernelGGL(k_point_rhs_set, dim3((nsrc + 255) / 256), dim3(256), 0, st, n, nsrc, nodes, amp, scale, b);
  return hipGetLastError();
}

hipError_t launch_gather(int nrhs, int nrec, const int* rec_nodes, const double2* u, size_t stride,
                         double2* d, hipStream_t st) {
  const int tot = nrhs * nrec;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((tot + 255) / 256), dim3(256), 0, st, nrhs, nrec, rec_nodes, u, stride, d);
  return hipGetLastError();
}

hipError_t launch_misfit(size_t nd, const double2* d_obs, const double2* d_cal, size_t nm,
                         const double* m, double lambda, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_misfit, dim3(1), dim3(1024), 0, st, nd, d_obs, d_cal, nm, m, lambda, out);
  return hipGetLastError();
}

hipError_t launch_inject(const Grid& gf, int dim, double* mc, hipStream_t st) {
  if (dim == 3) {
    const int tot = ((gf.nx + 1) / 2) * ((gf.ny + 1) / 2) * ((gf.nz + 1) / 2);
    hipLaunchKernelGGL(k_inject3, dim3((tot + 255) / 256), dim3(256), 0, st, gf, mc);
    return hipGetLastError();
  }
  const int ncx = (gf.nx + 1) / 2;
  const int ncz = dim == 2 ? (gf.nz + 1) / 2 : 1;
  const int tot = ncx * ncz;
  hipLaunchKernelGGL(k_inject, dim3((tot + 255) / 256), dim3(256), 0, st, gf, dim, mc);
  return hipGetLastError();
}

hipError_t launch_density_coef(const Grid& g, double* dc, hipStream_t st) {
  const size_t n = (size_t)g.nz * g.nx;
  if (!g.rho || g.ny != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_density_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, dc);
  return hipGetLastError();
}

hipError_t launch_check_density(size_t n, const double* m, const double* rho, double* out3, hipStream_t st) {
  hipLaunchKernelGGL(k_check_density, dim3(1), dim3(1024), 0, st, n, m, rho, out3);
  return hipGetLastError();
}

hipError_t launch_check_model(size_t n, const double* m, double* out3, hipStream_t st) {
  hipLaunchKernelGGL(k_check_model, dim3(1), dim3(1024), 0, st, n, m, out3);
  return hipGetLastError();
}

}  // namespace hz
