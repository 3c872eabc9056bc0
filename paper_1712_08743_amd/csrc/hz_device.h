// Device helpers shared by the HIP kernel files: complex arithmetic, the
// weighted Helmholtz stencil at one node, the mapping of blocks to (slot,
// tile), and fixed-order block reductions.
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
#pragma once

#include "hz_internal.h"

#include <math.h>

namespace hz {

// ---------------------------------------------------------------- complex helpers
__device__ __forceinline__ double2 c2(double a, double b) { return make_double2(a, b); }

// Streaming (non-temporal) 16-byte accesses for vectors a kernel touches once.
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(double2* p, double2 a) {
  d2v v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, reinterpret_cast<d2v*>(p));
}
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

// The slowness on grid g of the model that frequency entry f solves with.
__device__ __forceinline__ const double* model_m(const Grid& g, const FreqTab& f) {
  return g.m + (size_t)f.model * g.mstride;
}

struct NodeC {
  double wz, wx, lsum;
  double2 kap;
};

// ih = 1 / h of the node's level; gs scales the absorbing term (sqrt of the
// node's density under a variable density, see node_op).
template <bool D2>
__device__ __forceinline__ NodeC node_coef(int iz, int ix, int nz, int nx, double ih, double m,
                                           double omega, double s_re, double s_im, double gs = 1.0) {
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
  c.kap = c2(-om2wm2 * s_re, omega * g * m * ih * gs - om2wm2 * s_im);
  return c;
}

// (A x)_p from the value at p and the sum of its existing x- and
// z-neighbours (missing neighbours add nothing).
__device__ __forceinline__ double2 stencil(const NodeC& c, double ih2, double2 xp, double2 sx, double2 sz) {
  const double2 lx = c2(c.lsum * xp.x - c.wz * sx.x - c.wx * sz.x,
                        c.lsum * xp.y - c.wz * sx.y - c.wx * sz.y);
  return cadd(cscale(ih2, lx), cmul(c.kap, xp));
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
  return stencil(c, ih2, xp, sx, sz);
}

template <bool D2>
__device__ __forceinline__ double2 diag_of(const NodeC& c, double ih2) {
  return c2(c.lsum * ih2 + c.kap.x, c.kap.y);
}

// ---------------------------------------------------------------- variable density
// Eq. (1) with a density rho on the grid (Grid::rho): the coupling of node p
// with a neighbour q is the constant-density one times the density on their
// common face, (rho_p + rho_q) / 2; the absorbing term is written for the
// flux, rho du/dn + j omega m sqrt(rho) u = 0, so it carries sqrt(rho_p).
// With Grid::rho null node_op and apply_op are node_coef and apply_node.
struct NodeOp {
  NodeC c;       // lsum: the sum of the couplings in use
  double cq[4];  // density couplings to the -x, +x, -z, +z neighbours (0 where missing)
};

template <bool D2>
__device__ __forceinline__ NodeOp node_op(const Grid& g, int iz, int ix, int p, double m, double omega,
                                          double s_re, double s_im) {
  NodeOp o;
  if (!g.rho) {
    o.c = node_coef<D2>(iz, ix, g.nz, g.nx, 1.0 / g.h, m, omega, s_re, s_im);
    return o;
  }
  const double* r = g.rho;
  const double rp = r[p];
  o.c = node_coef<D2>(iz, ix, g.nz, g.nx, 1.0 / g.h, m, omega, s_re, s_im, sqrt(rp));
  o.cq[0] = ix > 0 ? o.c.wz * (0.5 * (rp + r[p - 1])) : 0.0;
  o.cq[1] = ix < g.nx - 1 ? o.c.wz * (0.5 * (rp + r[p + 1])) : 0.0;
  o.cq[2] = (D2 && iz > 0) ? o.c.wx * (0.5 * (rp + r[p - g.nx])) : 0.0;
  o.cq[3] = (D2 && iz < g.nz - 1) ? o.c.wx * (0.5 * (rp + r[p + g.nx])) : 0.0;
  o.c.lsum = (o.cq[0] + o.cq[1]) + (o.cq[2] + o.cq[3]);
  return o;
}

// (A x)_p with the value at p and the neighbours' values from val(dz, dx),
// which is called for the existing neighbours only.
template <bool D2, class F>
__device__ __forceinline__ double2 apply_op_at(const Grid& g, const NodeOp& o, int iz, int ix, double ih2,
                                               double2 xp, F val) {
  if (!g.rho) {
    double2 sx = c2(0.0, 0.0), sz = c2(0.0, 0.0);
    if (ix > 0) sx = cadd(sx, val(0, -1));
    if (ix < g.nx - 1) sx = cadd(sx, val(0, 1));
    if (D2) {
      if (iz > 0) sz = cadd(sz, val(-1, 0));
      if (iz < g.nz - 1) sz = cadd(sz, val(1, 0));
    }
    return stencil(o.c, ih2, xp, sx, sz);
  }
  double2 s = c2(0.0, 0.0);
  if (ix > 0) s = cadd(s, cscale(o.cq[0], val(0, -1)));
  if (ix < g.nx - 1) s = cadd(s, cscale(o.cq[1], val(0, 1)));
  if (D2) {
    if (iz > 0) s = cadd(s, cscale(o.cq[2], val(-1, 0)));
    if (iz < g.nz - 1) s = cadd(s, cscale(o.cq[3], val(1, 0)));
  }
  const double2 lx = c2(o.c.lsum * xp.x - s.x, o.c.lsum * xp.y - s.y);
  return cadd(cscale(ih2, lx), cmul(o.c.kap, xp));
}

// (A x)_p for x given at the slot's base pointer; xp = x[p].
template <bool D2>
__device__ __forceinline__ double2 apply_op(const Grid& g, const NodeOp& o, const double2* __restrict__ x, int p,
                                            int iz, int ix, double ih2, double2 xp) {
  if (!g.rho) return apply_node<D2>(x, p, iz, ix, g.nz, g.nx, ih2, o.c, xp);
  const int nx = g.nx;
  return apply_op_at<D2>(g, o, iz, ix, ih2, xp, [&](int dz, int dx) { return x[p + dz * nx + dx]; });
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

// Grid kernels over 2D tiles map blocks to XCDs: the hardware hands block b
// to XCD b % kXcd, so XCD x is given the x-th contiguous range of tile rows of
// every slot in turn. Its L2 then keeps that strip's coefficients (slowness,
// Jacobi weights) across slots, and the z-halo of a tile mostly comes from a
// tile the same XCD has just read. Grid size: tile_blocks(per_slot, cap).
constexpr int kXcd = 8;

__host__ __device__ __forceinline__ int xcd_chunk(int per_slot) { return (per_slot + kXcd - 1) / kXcd; }

__device__ __forceinline__ bool decode_tile(const Batch& bt, int per_slot, int& slot, int& tile) {
  const int bid = blockIdx.x;
  const int x = bid % kXcd, k = bid / kXcd;
  const int chunk = xcd_chunk(per_slot);
  const int si = k / chunk;
  tile = x * chunk + (k - si * chunk);
  if (tile >= per_slot || si >= *bt.nactive) return false;
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

// Per-slot reductions run in two kernels: every block of the producer stores
// its fixed-order block sum in partials[slot][tile][k], and a later kernel
// with one block per slot sums the tiles in tile order. Kernel boundaries
// make the partials visible; no device-scope fence is needed inside a kernel
// (such a fence writes back the L2 of the XCD, which is slow when the kernel
// streams large vectors). The order does not depend on scheduling or on the
// other slots of the batch, so results are bitwise batch-invariant.
template <int K>
__device__ __forceinline__ void store_partial(double (&v)[K], const Reduce& rd, int slot, int tile) {
  static_assert(K <= kPartialWidth, "partials hold kPartialWidth doubles per tile");
  block_sum<K>(v);
  if (threadIdx.x == 0) {
    double* dst = rd.partials + ((size_t)slot * rd.max_tiles + tile) * kPartialWidth;
#pragma unroll
    for (int k = 0; k < K; ++k) dst[k] = v[k];
  }
}

// Sum of the partials of one slot over `tiles` tiles; valid in thread 0.
template <int K>
__device__ __forceinline__ void sum_partials(double (&out)[K], const Reduce& rd, int slot, int tiles) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  const double* src = rd.partials + (size_t)slot * rd.max_tiles * kPartialWidth;
  for (int t = threadIdx.x; t < tiles; t += blockDim.x) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] += src[(size_t)t * kPartialWidth + k];
  }
  block_sum<K>(out);
}

// The active-list entry of a one-block-per-slot kernel, if its slot is active.
__device__ __forceinline__ bool decode_slot_block(const Batch& bt, int& slot) {
  const int si = blockIdx.x;
  if (si >= *bt.nactive) return false;
  slot = bt.active[si];
  return bt.slots[slot].status == kActive;
}

__device__ __forceinline__ size_t vec_index(int tile, int e) {
  return ((size_t)tile * kVecPerThread + e) * kBlock + threadIdx.x;
}

}  // namespace hz

namespace hz {

// ---------------------------------------------------------------- LDS tiles (2D)
// The right-hand side b of a V-cycle level, formed on the fly (MODE 0: read,
// MODE 1: BiCGSTAB p = r + beta (p_old - omega v), MODE 2: s = r - alpha v).
struct RhsIn {
  const double2* a;  // b (MODE 0) or r
  const double2* b;  // p_old (MODE 1, 4) or v (MODE 2)
  const double2* c;  // v (MODE 1); p^_old (MODE 4) or p^ (MODE 5), whose product with B is formed
};

template <int MODE>
__device__ __forceinline__ double2 rhs_at(const RhsIn& in, size_t q, double2 beta, double2 om,
                                          double2 al) {
  if (MODE == 0) return in.a[q];
  if (MODE == 1) return cadd(in.a[q], cmul(beta, csub(in.b[q], cmul(om, in.c[q]))));
  return csub(in.a[q], cmul(al, in.b[q]));
}

// A 256-thread block owns a kTX x kTZ tile of nodes; a radius-one stencil
// stage reads its input from an LDS copy of the tile plus a one-node halo
// (kHZ x kHX), filled once with coalesced row loads. Halo entries outside
// the grid hold zero, which is what a missing neighbour contributes (the
// node's own coupling sum lsum already leaves it out), so the stencil needs
// no boundary branches. Thread t handles the nodes (t / kTX + 4 r, t % kTX),
// r = 0 .. kTZ/4 - 1.
constexpr int kTX = 64, kTZ = 8;
constexpr int kHX = kTX + 2, kHZ = kTZ + 2;
constexpr int kRowsPerThread = kTZ * kTX / kBlock;

struct TileOrg {
  int z0, x0;  // first node of the tile
};

__device__ __forceinline__ TileOrg tile_org(int tile, int ntx) {
  const int tzi = tile / ntx;
  return TileOrg{tzi * kTZ, (tile - tzi * ntx) * kTX};
}

// S[hz][hx] = val(q) at grid node (z0 - 1 + hz, x0 - 1 + hx) if it exists, else 0;
// q is the node's index in the level's vectors (row pitch vpitch(g)).
template <class F>
__device__ __forceinline__ void fill_halo(double2 (*S)[kHX], const Grid& g, TileOrg t, F val) {
  const int vp = vpitch(g);
  for (int e = threadIdx.x; e < kHZ * kHX; e += kBlock) {
    const int hz = e / kHX, hx = e - hz * kHX;
    const int gz = t.z0 - 1 + hz, gx = t.x0 - 1 + hx;
    double2 v = make_double2(0.0, 0.0);
    if (gz >= 0 && gz < g.nz && gx >= 0 && gx < g.nx) v = val(gz * vp + gx, hz, hx);
    S[hz][hx] = v;
  }
}

// Neighbour sums of the node at tile position (lz, lx) from an LDS halo tile.
__device__ __forceinline__ void halo_sums(const double2 (*S)[kHX], int lz, int lx, double2& sx, double2& sz) {
  sx = cadd(S[lz + 1][lx], S[lz + 1][lx + 2]);
  sz = cadd(S[lz][lx + 1], S[lz + 2][lx + 1]);
}

// ---- lane exchange of the wavefront-marching kernels (lane = grid column)

// Neighbouring lanes' values by whole-wavefront DPP shifts (wave_shr:1,
// wave_shl:1 on the two 32-bit halves): VALU moves with a few cycles of
// latency, where a general shuffle goes through the LDS crossbar. The lane
// with no neighbour (0 from the left, 63 from the right) receives 0 (the
// bound control of the move).
constexpr int kDppWaveShr1 = 0x138;  // lane i takes lane i - 1
constexpr int kDppWaveShl1 = 0x130;  // lane i takes lane i + 1
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 from_left(double2 v) {  // value of lane - 1
  return make_double2(dpp_shift<kDppWaveShr1>(v.x), dpp_shift<kDppWaveShr1>(v.y));
}
__device__ __forceinline__ double2 from_right(double2 v) {  // value of lane + 1
  return make_double2(dpp_shift<kDppWaveShl1>(v.x), dpp_shift<kDppWaveShl1>(v.y));
}
// v where c holds, else zero (selected per component, so no stack copy is made)
__device__ __forceinline__ double2 keep(bool c, double2 v) {
  return make_double2(c ? v.x : 0.0, c ? v.y : 0.0);
}

// ---- variable density in the fused kernels (2D): Grid::dc holds, per level,
// three arrays of n: the coupling of each node to its right neighbour
// wz (rho_p + rho_right) / 2, to the neighbour below wx (rho_p + rho_below) / 2
// (zero where that neighbour is missing), and the absorbing term's weight
// g sqrt(rho_p) (see node_op). A node's coupling to its left (upper)
// neighbour is that neighbour's right (lower) one.
struct RhoC {
  double l, r, u, d;  // couplings to the left, right, upper and lower neighbour
};

// (M x)_p = [(l + r + u + d) x_p - (l x_l + r x_r + u x_u + d x_d)] / h^2 + kap x_p,
// kap = -omega^2 s w m^2 + j omega gb m / h with w = wx wz the mass weight;
// ka = -omega^2 Re s, kb = -omega^2 Im s, kc = omega / h
__device__ __forceinline__ double2 apply_m_rho(const RhoC& c, double gb, double w, double m, double ka, double kb,
                                               double kc, double ih2, double2 xp, double2 xl, double2 xr,
                                               double2 xu, double2 xd) {
  const double mw = w * (m * m);
  const double kre = ka * mw, kim = kb * mw + kc * gb * m;
  const double lsum = (c.l + c.r) + (c.u + c.d);
  const double sre = (c.l * xl.x + c.r * xr.x) + (c.u * xu.x + c.d * xd.x);
  const double sim = (c.l * xl.y + c.r * xr.y) + (c.u * xu.y + c.d * xd.y);
  return c2(ih2 * (lsum * xp.x - sre) + (kre * xp.x - kim * xp.y),
            ih2 * (lsum * xp.y - sim) + (kre * xp.y + kim * xp.x));
}

// One damped-Jacobi update in the form (1 - w) u + (w/D)(b + (sum of the
// couplings times the neighbours) / h^2), with density couplings.
__device__ __forceinline__ double2 jacobi_rho(double2 u, double2 b, double2 wd, const RhoC& c, double2 xl,
                                              double2 xr, double2 xu, double2 xd, double ih2, double omw) {
  const double tx = ih2 * ((c.l * xl.x + c.r * xr.x) + (c.u * xu.x + c.d * xd.x)) + b.x;
  const double ty = ih2 * ((c.l * xl.y + c.r * xr.y) + (c.u * xu.y + c.d * xd.y)) + b.y;
  return c2(omw * u.x + (wd.x * tx - wd.y * ty), omw * u.y + (wd.x * ty + wd.y * tx));
}

}  // namespace hz
