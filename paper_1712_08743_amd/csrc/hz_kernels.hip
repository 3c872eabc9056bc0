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

#include "hz_internal.h"

#include <math.h>

namespace hz {

// ---------------------------------------------------------------- complex helpers
__device__ __forceinline__ double2 c2(double a, double b) { return make_double2(a, b); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return c2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return c2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return c2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return c2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {
  return c2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cinv(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return c2(a.x / d, -a.y / d);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's scaling keeps the quotient accurate for badly scaled operands
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return c2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return c2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
__device__ __forceinline__ bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }
__device__ __forceinline__ bool czero(double2 a) { return a.x == 0.0 && a.y == 0.0; }

// ---------------------------------------------------------------- grid geometry
Tiles grid_tiles(int nz, int nx, int dim) {
  Tiles t;
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

int vec_tiles(size_t n) {
  const size_t per = (size_t)kBlock * kVecPerThread;
  return (int)((n + per - 1) / per);
}

struct NodeC {
  double wz, wx, lsum;
  double2 kap;
};

template <bool D2>
__device__ __forceinline__ NodeC node_coef(int iz, int ix, int nz, int nx, double h, double m,
                                           double omega, double s_re, double s_im) {
  NodeC c;
  const int x0 = (ix == 0), x1 = (ix == nx - 1);
  c.wx = (x0 | x1) ? 0.5 : 1.0;
  double g;
  if (D2) {
    const int z0 = (iz == 0), z1 = (iz == nz - 1);
    c.wz = (z0 | z1) ? 0.5 : 1.0;
    g = c.wz * (double)(x0 + x1) + c.wx * (double)(z0 + z1);
    c.lsum = c.wz * (double)(2 - x0 - x1) + c.wx * (double)(2 - z0 - z1);
  } else {
    c.wz = 1.0;
    g = (double)(x0 + x1);
    c.lsum = (double)(2 - x0 - x1);
  }
  const double om2wm2 = omega * omega * (c.wx * c.wz) * (m * m);
  c.kap = c2(-om2wm2 * s_re, omega * g * m / h - om2wm2 * s_im);
  return c;
}

// (A x)_p for x given at the slot's base pointer; xp = x[p].
template <bool D2>
__device__ __forceinline__ double2 apply_node(const double2* __restrict__ x, int p, int iz, int ix,
                                              int nz, int nx, double ih2, const NodeC& c,
                                              double2 xp) {
  double2 sx = c2(0.0, 0.0), sz = c2(0.0, 0.0);
  if (ix > 0) sx = cadd(sx, x[p - 1]);
  if (ix < nx - 1) sx = cadd(sx, x[p + 1]);
  if (D2) {
    if (iz > 0) sz = cadd(sz, x[p - nx]);
    if (iz < nz - 1) sz = cadd(sz, x[p + nx]);
  }
  const double2 lx = c2(c.lsum * xp.x - c.wz * sx.x - c.wx * sz.x,
                        c.lsum * xp.y - c.wz * sx.y - c.wx * sz.y);
  return cadd(cscale(ih2, lx), cmul(c.kap, xp));
}

template <bool D2>
__device__ __forceinline__ double2 diag_of(const NodeC& c, double ih2) {
  return c2(c.lsum * ih2 + c.kap.x, c.kap.y);
}

// Which block of the grid is this: active-list entry and tile.
__device__ __forceinline__ bool decode_block(const Batch& bt, int per_slot, int& slot, int& tile) {
  const int bid = blockIdx.x;
  const int si = bid / per_slot;
  tile = bid - si * per_slot;
  if (si >= *bt.nactive) return false;
  slot = bt.active[si];
  return bt.slots[slot].status == kActive;
}

template <bool D2>
__device__ __forceinline__ void tile_node(const Tiles& t, int tile, int& iz, int& ix) {
  const int tzi = tile / t.ntx;
  const int txi = tile - tzi * t.ntx;
  const int lid = threadIdx.x;
  const int lx = lid % t.tx;
  const int lz = lid / t.tx;
  ix = txi * t.tx + lx;
  iz = tzi * t.tz + lz;
  if (!D2) iz = 0;
}

// ---------------------------------------------------------------- reductions
// Sum K doubles over the block in a fixed order; the result is valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
  __shared__ double sh[K][kBlock / 64];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[k][w];
      v[k] = s;
    }
  }
}

// Per-slot reduction over `tiles` blocks. Each block stores its partial; the
// block that arrives last sums all partials in tile order (so the result does
// not depend on scheduling or on the batch) and returns true with the totals
// in thread 0's v. The counter is left at zero for the next kernel.
template <int K>
__device__ __forceinline__ bool finish_slot(double (&v)[K], const Reduce& rd, int slot, int tile,
                                            int tiles) {
  static_assert(K <= 4, "partials hold four doubles per tile");
  __shared__ int is_last;
  block_sum<K>(v);
  if (threadIdx.x == 0) {
    double* dst = rd.partials + ((size_t)slot * rd.max_tiles + tile) * 4;
#pragma unroll
    for (int k = 0; k < K; ++k) __hip_atomic_store(dst + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned old = __hip_atomic_fetch_add(rd.counters + slot, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
    is_last = (old == (unsigned)(tiles - 1));
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  const double* src = rd.partials + (size_t)slot * rd.max_tiles * 4;
  for (int t = threadIdx.x; t < tiles; t += blockDim.x) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      acc[k] += __hip_atomic_load(src + (size_t)t * 4 + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum<K>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = acc[k];
    __hip_atomic_store(rd.counters + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

// ---------------------------------------------------------------- stencil kernels
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_apply(Grid g, Tiles t, int lvl, int which, Batch bt,
                                                  const double2* __restrict__ x,
                                                  double2* __restrict__ y, size_t stride) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= g.nz || ix >= g.nx) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double sre = which ? f.sM_re : f.sB_re, sim = which ? f.sM_im : f.sB_im;
  const int p = iz * g.nx + ix;
  const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[p], f.omega, sre, sim);
  const double2* xs = x + (size_t)slot * stride;
  y[(size_t)slot * stride + p] = apply_node<D2>(xs, p, iz, ix, g.nz, g.nx, 1.0 / (g.h * g.h), c, xs[p]);
  (void)lvl;
}

// u_out = u_in + w (b - M u_in) / diag(M); ZERO: u_in = 0.
template <bool D2, bool ZERO>
__global__ void __launch_bounds__(kBlock) k_smooth(Grid g, Tiles t, int lvl, double w_override,
                                                   Batch bt, const double2* __restrict__ b,
                                                   const double2* __restrict__ u_in,
                                                   double2* __restrict__ u_out, size_t stride) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= g.nz || ix >= g.nx) return;
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const double w = w_override > 0.0 ? w_override : f.wj[lvl];
  const int p = iz * g.nx + ix;
  const double ih2 = 1.0 / (g.h * g.h);
  const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[p], f.omega, f.sM_re, f.sM_im);
  const double2 dinv = cinv(diag_of<D2>(c, ih2));
  const size_t base = (size_t)slot * stride;
  const double2 bp = b[base + p];
  double2 out;
  if (ZERO) {
    out = cscale(w, cmul(bp, dinv));
  } else {
    const double2* us = u_in + base;
    const double2 up = us[p];
    const double2 res = csub(bp, apply_node<D2>(us, p, iz, ix, g.nz, g.nx, ih2, c, up));
    out = cadd(up, cscale(w, cmul(res, dinv)));
  }
  u_out[base + p] = out;
}

// bc = 2^-dim P^T (b - M u), one thread per coarse node.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_restrict(Grid gf, Grid gc, Tiles t, Batch bt,
                                                     const double2* __restrict__ b,
                                                     const double2* __restrict__ u,
                                                     double2* __restrict__ bc, size_t sf,
                                                     size_t sc) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
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
    const double wzt = (dz == 0) ? 1.0 : 0.5;
    double2 row = c2(0.0, 0.0);
    for (int dx = -1; dx <= 1; ++dx) {
      const int ix = 2 * Ix + dx;
      if (ix < 0 || ix >= gf.nx) continue;
      const int p = iz * gf.nx + ix;
      const NodeC c = node_coef<D2>(iz, ix, gf.nz, gf.nx, gf.h, gf.m[p], f.omega, f.sM_re, f.sM_im);
      const double2 r = csub(bs[p], apply_node<D2>(us, p, iz, ix, gf.nz, gf.nx, ih2, c, us[p]));
      const double wxt = (dx == 0) ? 1.0 : 0.5;
      row = cadd(row, cscale(wxt, r));
    }
    acc = cadd(acc, cscale(wzt, row));
  }
  bc[(size_t)slot * sc + Iz * gc.nx + Ix] = cscale(D2 ? 0.25 : 0.5, acc);
}

// Bilinear (1D: linear) interpolation of coarse e at fine node (iz, ix).
template <bool D2>
__device__ __forceinline__ double2 interp(const double2* __restrict__ e, int iz, int ix, int ncx) {
  const int Jx = ix >> 1, ox = ix & 1;
  if (!D2) {
    return ox ? cscale(0.5, cadd(e[Jx], e[Jx + 1])) : e[Jx];
  }
  const int Jz = iz >> 1, oz = iz & 1;
  const double2* r0 = e + Jz * ncx;
  double2 a = ox ? cscale(0.5, cadd(r0[Jx], r0[Jx + 1])) : r0[Jx];
  if (!oz) return a;
  const double2* r1 = r0 + ncx;
  const double2 bb = ox ? cscale(0.5, cadd(r1[Jx], r1[Jx + 1])) : r1[Jx];
  return cscale(0.5, cadd(a, bb));
}

// u_out = u_in + P e (u_out may be u_in: each thread reads, then writes, its own node).
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_prolong(Grid gf, Grid gc, Tiles t, Batch bt,
                                                    const double2* __restrict__ e,
                                                    const double2* u_in, double2* u_out,
                                                    size_t sf, size_t sc) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  if (iz >= gf.nz || ix >= gf.nx) return;
  const size_t q = (size_t)slot * sf + iz * gf.nx + ix;
  const double2 ef = interp<D2>(e + (size_t)slot * sc, iz, ix, gc.nx);
  u_out[q] = cadd(u_in[q], ef);
}

// ---------------------------------------------------------------- coarse solve
// uc[slot] = Cinv_f bc[slot]. Cinv is symmetric (M is complex symmetric), so
// the row needed by thread `row` is read as a column: Cinv[k][row], which is
// coalesced across the block. Each block takes up to kCoarseGroup consecutive
// active slots (consecutive slots share a frequency except at group borders,
// handled by segments).
__global__ void __launch_bounds__(kCoarseRows) k_coarse(int nc, Batch bt,
                                                        const double2* __restrict__ bc,
                                                        double2* __restrict__ uc, size_t stride) {
  __shared__ double2 bsh[kCoarseGroup][kCoarseRows];
  __shared__ int sslot[kCoarseGroup], sfreq[kCoarseGroup];
  const int na = *bt.nactive;
  const int base = blockIdx.y * kCoarseGroup;
  if (base >= na) return;
  const int cnt = min(kCoarseGroup, na - base);
  if (threadIdx.x < kCoarseGroup) {
    const int j = threadIdx.x;
    if (j < cnt) {
      sslot[j] = bt.active[base + j];
      sfreq[j] = bt.slots[sslot[j]].freq;
    } else {
      sslot[j] = -1;
      sfreq[j] = -1;
    }
  }
  __syncthreads();
  const int row = blockIdx.x * kCoarseRows + threadIdx.x;
  int j0 = 0;
  while (j0 < cnt) {
    const int fq = sfreq[j0];
    int j1 = j0;
    while (j1 < cnt && sfreq[j1] == fq) ++j1;
    const double2* Ci = bt.ft[fq].cinv;
    double2 acc[kCoarseGroup];
#pragma unroll
    for (int j = 0; j < kCoarseGroup; ++j) acc[j] = c2(0.0, 0.0);
    for (int k0 = 0; k0 < nc; k0 += kCoarseRows) {
      const int kk = k0 + threadIdx.x;
#pragma unroll
      for (int j = 0; j < kCoarseGroup; ++j) {
        double2 val = c2(0.0, 0.0);
        if (j >= j0 && j < j1 && kk < nc) val = bc[(size_t)sslot[j] * stride + kk];
        bsh[j][threadIdx.x] = val;
      }
      __syncthreads();
      if (row < nc) {
        const int kend = min(kCoarseRows, nc - k0);
        const double2* col = Ci + (size_t)k0 * nc + row;
        for (int q = 0; q < kend; ++q) {
          const double2 a = col[(size_t)q * nc];
#pragma unroll
          for (int j = 0; j < kCoarseGroup; ++j) {
            const double2 bv = bsh[j][q];
            acc[j].x += a.x * bv.x - a.y * bv.y;
            acc[j].y += a.x * bv.y + a.y * bv.x;
          }
        }
      }
      __syncthreads();
    }
    if (row < nc) {
      for (int j = j0; j < j1; ++j) uc[(size_t)sslot[j] * stride + row] = acc[j];
    }
    j0 = j1;
  }
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
    const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[i], ft[f].omega, ft[f].sM_re, ft[f].sM_im);
    double2 val = c2(0.0, 0.0);
    if (i == j) {
      val = diag_of<D2>(c, ih2);
    } else if (jz == iz && (jx == ix - 1 || jx == ix + 1)) {
      val = c2(-c.wz * ih2, 0.0);
    } else if (D2 && jx == ix && (jz == iz - 1 || jz == iz + 1)) {
      val = c2(-c.wx * ih2, 0.0);
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
    const NodeC c = node_coef<false>(0, i, 1, n, g.h, g.m[i], f.omega, f.sM_re, f.sM_im);
    A[i] = c2(i > 0 ? -ih2 : 0.0, 0.0);
    Cu[i] = c2(i < n - 1 ? -ih2 : 0.0, 0.0);
    Bd[i] = diag_of<false>(c, ih2);
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

// ---------------------------------------------------------------- pointwise helpers
__device__ __forceinline__ bool decode_vec(const Batch& bt, int tiles, int& slot, int& tile) {
  return decode_block(bt, tiles, slot, tile);
}

__global__ void __launch_bounds__(kBlock) k_copy(Batch bt, int tiles, size_t n,
                                                 const double2* __restrict__ x,
                                                 double2* __restrict__ y, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) y[base + i] = x[base + i];
  }
}

// x = 0, r = rh = b, p = v = 0; ||b||^2 -> initial scalars.
__global__ void __launch_bounds__(kBlock) k_bicg_init(Batch bt, int tiles, size_t n, Reduce rd,
                                                      const double2* __restrict__ b,
                                                      double2* __restrict__ x, double2* __restrict__ r,
                                                      double2* __restrict__ rh, double2* __restrict__ p,
                                                      double2* __restrict__ v, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) {
      const double2 bi = b[base + i];
      const double2 z = c2(0.0, 0.0);
      x[base + i] = z;
      r[base + i] = bi;
      rh[base + i] = bi;
      p[base + i] = z;
      v[base + i] = z;
      acc[0] += bi.x * bi.x + bi.y * bi.y;
    }
  }
  if (finish_slot<1>(acc, rd, slot, tile, tiles) && threadIdx.x == 0) {
    Slot& S = bt.slots[slot];
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
      // first step: rho' = <rhat, r> = ||b||^2, beta = (rho'/1)(1/1)
      S.rho = c2(b2, 0.0);
      S.beta = c2(b2, 0.0);
    }
  }
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(kBlock) k_bicg_p(Batch bt, int tiles, size_t n,
                                                   const double2* __restrict__ r,
                                                   double2* __restrict__ p,
                                                   const double2* __restrict__ v, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const Slot& S = bt.slots[slot];
  const double2 beta = S.beta, om = S.omega;
  const size_t base = (size_t)slot * stride;
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) {
      const double2 t = csub(p[base + i], cmul(om, v[base + i]));
      p[base + i] = cadd(r[base + i], cmul(beta, t));
    }
  }
}

// v = B ph; sigma = <rh, v>; alpha = rho / sigma.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_bicg_apply_sigma(Grid g, Tiles t, Batch bt, Reduce rd,
                                                             const double2* __restrict__ ph,
                                                             const double2* __restrict__ rh,
                                                             double2* __restrict__ v, size_t stride) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[p], f.omega, f.sB_re, f.sB_im);
    const double2* xs = ph + base;
    const double2 y = apply_node<D2>(xs, p, iz, ix, g.nz, g.nx, 1.0 / (g.h * g.h), c, xs[p]);
    v[base + p] = y;
    const double2 d = cconjmul(rh[base + p], y);
    acc[0] = d.x;
    acc[1] = d.y;
  }
  if (finish_slot<2>(acc, rd, slot, tile, t.per_slot) && threadIdx.x == 0) {
    Slot& S = bt.slots[slot];
    const double2 sigma = c2(acc[0], acc[1]);
    if (!cfinite(sigma)) {
      S.status = kNonfinite;
    } else if (czero(sigma)) {
      S.status = S.restarted ? kBreakdown : kRestart;
    } else {
      S.alpha = cdiv(S.rho, sigma);
    }
  }
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
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) s[base + i] = csub(r[base + i], cmul(al, v[base + i]));
  }
}

// t = B sh; omega = <t, s> / <t, t>.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_bicg_apply_omega(Grid g, Tiles t, Batch bt, Reduce rd,
                                                             const double2* __restrict__ sh,
                                                             const double2* __restrict__ s,
                                                             double2* __restrict__ tv, size_t stride) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[3] = {0.0, 0.0, 0.0};
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[p], f.omega, f.sB_re, f.sB_im);
    const double2* xs = sh + base;
    const double2 y = apply_node<D2>(xs, p, iz, ix, g.nz, g.nx, 1.0 / (g.h * g.h), c, xs[p]);
    tv[base + p] = y;
    const double2 ts = cconjmul(y, s[base + p]);
    acc[0] = ts.x;
    acc[1] = ts.y;
    acc[2] = y.x * y.x + y.y * y.y;
  }
  if (finish_slot<3>(acc, rd, slot, tile, t.per_slot) && threadIdx.x == 0) {
    Slot& S = bt.slots[slot];
    const double tt = acc[2];
    const double2 om = tt != 0.0 ? c2(acc[0] / tt, acc[1] / tt) : c2(0.0, 0.0);
    if (!cfinite(S.alpha) || !cfinite(om)) {
      S.status = kNonfinite;
    } else {
      S.omega = om;
    }
  }
}

// x += alpha ph + omega sh; r = s - omega t; then the step's end: convergence,
// restart or breakdown, and the next step's rho and beta from <rh, r>.
__global__ void __launch_bounds__(kBlock) k_bicg_xr(Batch bt, int tiles, size_t n, Reduce rd,
                                                    double tol, int maxit, double2* __restrict__ x,
                                                    const double2* __restrict__ ph,
                                                    const double2* __restrict__ sh,
                                                    const double2* __restrict__ s,
                                                    const double2* __restrict__ t,
                                                    double2* __restrict__ r,
                                                    const double2* __restrict__ rh, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const Slot& S0 = bt.slots[slot];
  const double2 al = S0.alpha, om = S0.omega;
  const size_t base = (size_t)slot * stride;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) {
      const size_t q = base + i;
      x[q] = cadd(x[q], cadd(cmul(al, ph[q]), cmul(om, sh[q])));
      const double2 ri = csub(s[q], cmul(om, t[q]));
      r[q] = ri;
      const double2 d = cconjmul(rh[q], ri);
      acc[0] += d.x;
      acc[1] += d.y;
      acc[2] += ri.x * ri.x + ri.y * ri.y;
    }
  }
  if (finish_slot<3>(acc, rd, slot, tile, tiles) && threadIdx.x == 0) {
    Slot& S = bt.slots[slot];
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
    } else if (czero(rho_new)) {
      S.status = S.restarted ? kBreakdown : kRestart;
    } else {
      S.beta = cmul(cdiv(rho_new, S.rho), cdiv(S.alpha, S.omega));
      S.rho = rho_new;
    }
  }
}

// The one restart after a breakdown: rh = r, p = v = 0, rho = <r, r>, beta = rho.
__global__ void __launch_bounds__(kBlock) k_bicg_restart(int tiles, size_t n, Batch bt, Reduce rd,
                                                         const double2* __restrict__ r,
                                                         double2* __restrict__ rh,
                                                         double2* __restrict__ p,
                                                         double2* __restrict__ v, size_t stride) {
  const int slot = blockIdx.x / tiles;
  const int tile = blockIdx.x - slot * tiles;
  if (bt.slots[slot].status != kRestart) return;
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) {
      const double2 ri = r[base + i];
      rh[base + i] = ri;
      p[base + i] = c2(0.0, 0.0);
      v[base + i] = c2(0.0, 0.0);
      const double2 d = cconjmul(ri, ri);
      acc[0] += d.x;
      acc[1] += d.y;
    }
  }
  if (finish_slot<2>(acc, rd, slot, tile, tiles) && threadIdx.x == 0) {
    Slot& S = bt.slots[slot];
    const double2 rho = c2(acc[0], acc[1]);
    S.restarted = 1;
    S.alpha = c2(1.0, 0.0);
    S.omega = c2(1.0, 0.0);
    if (!cfinite(rho)) {
      S.status = kNonfinite;
    } else if (czero(rho)) {
      S.status = kBreakdown;
    } else {
      S.rho = rho;
      S.beta = rho;
      S.status = kActive;
    }
  }
}

// Rebuild the active list (ascending slot ids) and the host summary.
__global__ void __launch_bounds__(1024) k_compact(int nslots, const Slot* __restrict__ slots,
                                                  int* __restrict__ active, int* __restrict__ nactive,
                                                  Summary* sum, int want_phase) {
  __shared__ int wsum[16];
  __shared__ int wres[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  int nres_local = 0, noth_local = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nslots; b0 += blockDim.x) {
    const int i = b0 + threadIdx.x;
    const int st = i < nslots ? slots[i].status : kConverged;
    const int ph = i < nslots ? slots[i].phase : 0;
    const int a = (st == kActive) && (ph == want_phase);
    nres_local += (st == kRestart);
    noth_local += (st == kActive) && (ph != want_phase);
    // inclusive scan of a over the block
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = a;
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
  // restart-pending and other-phase counts
  __shared__ int woth[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    nres_local += __shfl_xor(nres_local, off, 64);
    noth_local += __shfl_xor(noth_local, off, 64);
  }
  if (lane == 0) {
    wres[wid] = nres_local;
    woth[wid] = noth_local;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nr = 0, no = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      nr += wres[w];
      no += woth[w];
    }
    *nactive = carry;
    sum->nactive = carry;
    sum->nrestart = nr;
    sum->nother = no;
  }
}

// ||b - B x||^2 and ||b||^2 per slot.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_true_residual(Grid g, Tiles t, Batch bt, Reduce rd,
                                                          const double2* __restrict__ b,
                                                          const double2* __restrict__ x,
                                                          double* __restrict__ out, size_t stride) {
  const int si = blockIdx.x / t.per_slot;
  const int tile = blockIdx.x - si * t.per_slot;
  if (si >= *bt.nactive) return;
  const int slot = bt.active[si];
  int iz, ix;
  tile_node<D2>(t, tile, iz, ix);
  const FreqTab& f = bt.ft[bt.slots[slot].freq];
  const size_t base = (size_t)slot * stride;
  double acc[2] = {0.0, 0.0};
  if (iz < g.nz && ix < g.nx) {
    const int p = iz * g.nx + ix;
    const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[p], f.omega, f.sB_re, f.sB_im);
    const double2* xs = x + base;
    const double2 y = apply_node<D2>(xs, p, iz, ix, g.nz, g.nx, 1.0 / (g.h * g.h), c, xs[p]);
    const double2 bp = b[base + p];
    const double2 rr = csub(bp, y);
    acc[0] = rr.x * rr.x + rr.y * rr.y;
    acc[1] = bp.x * bp.x + bp.y * bp.y;
  }
  if (finish_slot<2>(acc, rd, slot, tile, t.per_slot) && threadIdx.x == 0) {
    out[2 * slot] = acc[0];
    out[2 * slot + 1] = acc[1];
  }
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
  const int ncx = (gf.nx - 1) / 2 + 1;
  const int ncz = dim == 2 ? (gf.nz - 1) / 2 + 1 : 1;
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

// ---------------------------------------------------------------- GMRES(m)
// Right-preconditioned restarted GMRES, one Arnoldi process per slot, all
// slots of a cycle in lockstep. The basis vector i of slot s lives at
// V + i * vstride + s * stride. Orthogonalisation is classical Gram-Schmidt
// applied twice; every per-slot sum is a fixed-order reduction.

// r = b - B x (x = 0 on the first cycle, which also zeroes x) into V_0, and
// the cycle start: beta = ||r||, g = (beta, 0, ...), or a final status.
template <bool D2>
__global__ void __launch_bounds__(kBlock) k_gm_residual(Grid g, Tiles t, Batch bt, Reduce rd, Gmres gm,
                                                        int first, double tol, int maxit,
                                                        const double2* __restrict__ b,
                                                        double2* __restrict__ x,
                                                        double2* __restrict__ v0, size_t stride) {
  int slot, tile;
  if (!decode_block(bt, t.per_slot, slot, tile)) return;
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
      const NodeC c = node_coef<D2>(iz, ix, g.nz, g.nx, g.h, g.m[p], f.omega, f.sB_re, f.sB_im);
      const double2* xs = x + base;
      r = csub(b[base + p], apply_node<D2>(xs, p, iz, ix, g.nz, g.nx, 1.0 / (g.h * g.h), c, xs[p]));
    }
    v0[base + p] = r;
    acc[0] = r.x * r.x + r.y * r.y;
  }
  if (finish_slot<1>(acc, rd, slot, tile, t.per_slot) && threadIdx.x == 0) {
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
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) v[base + i] = cscale(inv, v[base + i]);
  }
}

// h_i = <V_i, w>, i = 0..j, into hc[pass]; pass 0 sets column j of H, pass 1 adds.
__global__ void __launch_bounds__(kBlock) k_gm_dots(Batch bt, int tiles, size_t n, Reduce rd, Gmres gm,
                                                    int j, int pass, const double2* __restrict__ V,
                                                    size_t vstride, const double2* __restrict__ w,
                                                    size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
  const int nv = j + 1;
  const int width = 2 * (gm.m + 1);
  double* part = gm.partials + ((size_t)slot * gm.max_tiles + tile) * width;
  for (int c0 = 0; c0 < nv; c0 += 8) {
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
#pragma unroll
    for (int e = 0; e < kVecPerThread; ++e) {
      const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
      if (i < n) {
        const double2 wi = w[base + i];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (c0 + q < nv) {
            const double2 d = cconjmul(V[(size_t)(c0 + q) * vstride + base + i], wi);
            acc[2 * q] += d.x;
            acc[2 * q + 1] += d.y;
          }
        }
      }
    }
    block_sum<16>(acc);
    if (threadIdx.x == 0) {
      for (int q = 0; q < 8 && c0 + q < nv; ++q) {
        __hip_atomic_store(part + 2 * (c0 + q), acc[2 * q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(part + 2 * (c0 + q) + 1, acc[2 * q + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __shared__ int is_last;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned old = __hip_atomic_fetch_add(rd.counters + slot, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (old == (unsigned)(tiles - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const double* src = gm.partials + (size_t)slot * gm.max_tiles * width;
  double2* hc = gm.hc + ((size_t)slot * 2 + pass) * (gm.m + 1);
  double2* Hc = gm.H + (size_t)slot * (gm.m + 1) * gm.m + (size_t)j * (gm.m + 1);
  for (int v = threadIdx.x; v < 2 * nv; v += blockDim.x) {
    double sum = 0.0;
    for (int tt = 0; tt < tiles; ++tt)
      sum += __hip_atomic_load(src + (size_t)tt * width + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int i = v >> 1;
    if (v & 1) {
      hc[i].y = sum;
      Hc[i].y = pass ? Hc[i].y + sum : sum;
    } else {
      hc[i].x = sum;
      Hc[i].x = pass ? Hc[i].x + sum : sum;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(rd.counters + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// w -= sum_i hc[pass]_i V_i. After the second pass: ||w|| becomes H[j+1, j],
// the new rotation is formed and the cycle-end test is made.
__global__ void __launch_bounds__(kBlock) k_gm_orth(Batch bt, int tiles, size_t n, Reduce rd, Gmres gm,
                                                    int j, int pass, double tol, int maxit,
                                                    const double2* __restrict__ V, size_t vstride,
                                                    double2* __restrict__ w, size_t stride) {
  int slot, tile;
  if (!decode_vec(bt, tiles, slot, tile)) return;
  const size_t base = (size_t)slot * stride;
  const double2* hc = gm.hc + ((size_t)slot * 2 + pass) * (gm.m + 1);
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < kVecPerThread; ++e) {
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) {
      double2 wi = w[base + i];
      for (int q = 0; q <= j; ++q) wi = csub(wi, cmul(hc[q], V[(size_t)q * vstride + base + i]));
      w[base + i] = wi;
      acc[0] += wi.x * wi.x + wi.y * wi.y;
    }
  }
  if (!pass) return;
  if (finish_slot<1>(acc, rd, slot, tile, tiles) && threadIdx.x == 0) {
    Slot& S = bt.slots[slot];
    const int m1 = gm.m + 1;
    double2* Hc = gm.H + (size_t)slot * m1 * gm.m + (size_t)j * m1;
    double* cs = gm.cs + (size_t)slot * gm.m;
    double2* sn = gm.sn + (size_t)slot * gm.m;
    double2* gg = gm.g + (size_t)slot * m1;
    const double nrm = sqrt(acc[0]);
    Hc[j + 1] = c2(nrm, 0.0);
    for (int i = 0; i < j; ++i) {
      const double2 a = Hc[i], bb = Hc[i + 1];
      Hc[i] = cadd(cscale(cs[i], a), cmul(sn[i], bb));
      Hc[i + 1] = csub(cscale(cs[i], bb), cmul(c2(sn[i].x, -sn[i].y), a));
    }
    double cj;
    double2 sj;
    givens(Hc[j], Hc[j + 1], cj, sj);
    cs[j] = cj;
    sn[j] = sj;
    Hc[j] = cadd(cscale(cj, Hc[j]), cmul(sj, Hc[j + 1]));
    Hc[j + 1] = c2(0.0, 0.0);
    const double2 gj = gg[j];
    gg[j + 1] = cmul(c2(-sj.x, sj.y), gj);  // -conj(s) g_j
    gg[j] = cscale(cj, gj);
    S.iters += 1;
    S.cyc_k = j + 1;
    S.t1 = wall_clock64();
    S.scal = c2(nrm, 0.0);
    const double est = sqrt(gg[j + 1].x * gg[j + 1].x + gg[j + 1].y * gg[j + 1].y);
    if (!isfinite(est) || !isfinite(nrm)) {
      S.status = kNonfinite;
    } else if (est <= tol * sqrt(S.bnorm2) || S.iters >= maxit || j + 1 == gm.m) {
      S.phase = 1;
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
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
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
    const size_t i = ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
    if (i < n) x[base + i] = cadd(x[base + i], z[base + i]);
  }
}

// ---------------------------------------------------------------- launchers
static inline dim3 grid1(long long blocks) { return dim3((unsigned)blocks); }

hipError_t launch_apply(int dim, const Grid& g, int lvl, int which, const Batch& bt, int cap,
                        const double2* x, double2* y, size_t stride, hipStream_t st) {
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(k_apply<true>, grid1((long long)cap * t.per_slot), dim3(kBlock), 0, st, g, t, lvl, which, bt, x, y, stride);
  else
    hipLaunchKernelGGL(k_apply<false>, grid1((long long)cap * t.per_slot), dim3(kBlock), 0, st, g, t, lvl, which, bt, x, y, stride);
  return hipGetLastError();
}

hipError_t launch_smooth(int dim, const Grid& g, int lvl, double w_override, const Batch& bt,
                         int cap, const double2* b, const double2* u_in, double2* u_out,
                         size_t stride, hipStream_t st) {
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * t.per_slot);
  if (dim == 2) {
    if (u_in)
      hipLaunchKernelGGL((k_smooth<true, false>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride);
    else
      hipLaunchKernelGGL((k_smooth<true, true>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride);
  } else {
    if (u_in)
      hipLaunchKernelGGL((k_smooth<false, false>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride);
    else
      hipLaunchKernelGGL((k_smooth<false, true>), gr, dim3(kBlock), 0, st, g, t, lvl, w_override, bt, b, u_in, u_out, stride);
  }
  return hipGetLastError();
}

hipError_t launch_restrict(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                           const double2* b, const double2* u, double2* bc, size_t sf, size_t sc,
                           hipStream_t st) {
  const Tiles t = grid_tiles(gc.nz, gc.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * t.per_slot);
  if (dim == 2)
    hipLaunchKernelGGL(k_restrict<true>, gr, dim3(kBlock), 0, st, gf, gc, t, bt, b, u, bc, sf, sc);
  else
    hipLaunchKernelGGL(k_restrict<false>, gr, dim3(kBlock), 0, st, gf, gc, t, bt, b, u, bc, sf, sc);
  return hipGetLastError();
}

hipError_t launch_prolong(int dim, const Grid& gf, const Grid& gc, const Batch& bt, int cap,
                          const double2* e, const double2* u_in, double2* u_out, size_t sf,
                          size_t sc, hipStream_t st) {
  const Tiles t = grid_tiles(gf.nz, gf.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * t.per_slot);
  if (dim == 2)
    hipLaunchKernelGGL(k_prolong<true>, gr, dim3(kBlock), 0, st, gf, gc, t, bt, e, u_in, u_out, sf, sc);
  else
    hipLaunchKernelGGL(k_prolong<false>, gr, dim3(kBlock), 0, st, gf, gc, t, bt, e, u_in, u_out, sf, sc);
  return hipGetLastError();
}

hipError_t launch_coarse_solve(int nc, const Batch& bt, int cap, const double2* bc, double2* uc,
                               size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const dim3 gr((nc + kCoarseRows - 1) / kCoarseRows, (cap + kCoarseGroup - 1) / kCoarseGroup);
  hipLaunchKernelGGL(k_coarse, gr, dim3(kCoarseRows), 0, st, nc, bt, bc, uc, stride);
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

hipError_t launch_copy(const Batch& bt, int cap, size_t n, const double2* x, double2* y,
                       size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_copy, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, x, y, stride);
  return hipGetLastError();
}

static inline unsigned flat_blocks(size_t total) {
  size_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return (unsigned)b;
}

hipError_t launch_assemble_dense(int dim, const Grid& g, int nfreq, const FreqTab* ft, double2* A,
                                 hipStream_t st) {
  const size_t nc = (size_t)g.nz * g.nx;
  const unsigned nb = flat_blocks(nc * nc * nfreq);
  if (dim == 2)
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

hipError_t launch_bicg_init(size_t n, const Batch& bt, int cap, const Reduce& rd, const double2* b,
                            double2* x, double2* r, double2* rh, double2* p, double2* v,
                            size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_init, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, rd, b, x, r, rh, p, v, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_p(size_t n, const Batch& bt, int cap, const double2* r, double2* p,
                         const double2* v, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_p, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, r, p, v, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_apply_sigma(int dim, const Grid& g, const Batch& bt, int cap,
                                   const Reduce& rd, const double2* ph, const double2* rh,
                                   double2* v, size_t stride, hipStream_t st) {
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * t.per_slot);
  if (dim == 2)
    hipLaunchKernelGGL(k_bicg_apply_sigma<true>, gr, dim3(kBlock), 0, st, g, t, bt, rd, ph, rh, v, stride);
  else
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
  const Tiles tl = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * tl.per_slot);
  if (dim == 2)
    hipLaunchKernelGGL(k_bicg_apply_omega<true>, gr, dim3(kBlock), 0, st, g, tl, bt, rd, sh, s, t, stride);
  else
    hipLaunchKernelGGL(k_bicg_apply_omega<false>, gr, dim3(kBlock), 0, st, g, tl, bt, rd, sh, s, t, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_xr(size_t n, const Batch& bt, int cap, const Reduce& rd, double tol,
                          int maxit, double2* x, const double2* ph, const double2* sh,
                          const double2* s, const double2* t, double2* r, const double2* rh,
                          size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_xr, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, rd, tol, maxit, x, ph, sh, s, t, r, rh, stride);
  return hipGetLastError();
}

hipError_t launch_bicg_restart(size_t n, int nslots, const Batch& bt, const Reduce& rd,
                               const double2* r, double2* rh, double2* p, double2* v,
                               size_t stride, hipStream_t st) {
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_bicg_restart, grid1((long long)nslots * tiles), dim3(kBlock), 0, st, tiles, n, bt, rd, r, rh, p, v, stride);
  return hipGetLastError();
}

hipError_t launch_compact(int nslots, Slot* slots, int* active, int* nactive, Summary* sum,
                          int want_phase, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, nslots, slots, active, nactive, sum, want_phase);
  return hipGetLastError();
}

hipError_t launch_true_residual(int dim, const Grid& g, const Batch& bt, int cap, const Reduce& rd,
                                const double2* b, const double2* x, double* out, size_t stride,
                                hipStream_t st) {
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * t.per_slot);
  if (dim == 2)
    hipLaunchKernelGGL(k_true_residual<true>, gr, dim3(kBlock), 0, st, g, t, bt, rd, b, x, out, stride);
  else
    hipLaunchKernelGGL(k_true_residual<false>, gr, dim3(kBlock), 0, st, g, t, bt, rd, b, x, out, stride);
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
  const int ncx = (gf.nx - 1) / 2 + 1;
  const int ncz = dim == 2 ? (gf.nz - 1) / 2 + 1 : 1;
  const int tot = ncx * ncz;
  hipLaunchKernelGGL(k_inject, dim3((tot + 255) / 256), dim3(256), 0, st, gf, dim, mc);
  return hipGetLastError();
}

hipError_t launch_check_model(size_t n, const double* m, double* out3, hipStream_t st) {
  hipLaunchKernelGGL(k_check_model, dim3(1), dim3(1024), 0, st, n, m, out3);
  return hipGetLastError();
}

hipError_t launch_gm_residual(int dim, const Grid& g, const Batch& bt, int cap, const Reduce& rd,
                              const Gmres& gm, int first, double tol, int maxit, const double2* b,
                              const double2* x, double2* v0, size_t stride, hipStream_t st) {
  const Tiles t = grid_tiles(g.nz, g.nx, dim);
  if (cap <= 0) return hipSuccess;
  const dim3 gr = grid1((long long)cap * t.per_slot);
  double2* xx = const_cast<double2*>(x);
  if (dim == 2)
    hipLaunchKernelGGL(k_gm_residual<true>, gr, dim3(kBlock), 0, st, g, t, bt, rd, gm, first, tol, maxit, b, xx, v0, stride);
  else
    hipLaunchKernelGGL(k_gm_residual<false>, gr, dim3(kBlock), 0, st, g, t, bt, rd, gm, first, tol, maxit, b, xx, v0, stride);
  return hipGetLastError();
}

hipError_t launch_gm_scale(size_t n, const Batch& bt, int cap, double2* v, size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_gm_scale, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, v, stride);
  return hipGetLastError();
}

hipError_t launch_gm_dots(size_t n, const Batch& bt, int cap, const Reduce& rd, const Gmres& gm, int j,
                          int pass, const double2* V, size_t vstride, const double2* w, size_t stride,
                          hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_gm_dots, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, rd, gm, j, pass, V, vstride, w, stride);
  return hipGetLastError();
}

hipError_t launch_gm_orth(size_t n, const Batch& bt, int cap, const Reduce& rd, const Gmres& gm, int j,
                          int pass, double tol, int maxit, const double2* V, size_t vstride, double2* w,
                          size_t stride, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int tiles = vec_tiles(n);
  hipLaunchKernelGGL(k_gm_orth, grid1((long long)cap * tiles), dim3(kBlock), 0, st, bt, tiles, n, rd, gm, j, pass, tol, maxit, V, vstride, w, stride);
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
