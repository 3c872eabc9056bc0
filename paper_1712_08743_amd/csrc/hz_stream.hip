// Wave-streaming forms of the two fused V-cycle kernels on 2D grids.
//
// One wavefront owns a strip of 64 consecutive columns (lane = column) and a
// chunk of rows of one right-hand side, and marches down the rows. Each
// stage of a kernel runs a fixed number of rows behind the stage it reads,
// so the z-neighbours of a node are values the lane computed in the last
// few rows and keeps in registers; x-neighbours come from the adjacent lanes
// through cross-lane moves. There is no LDS staging and no barrier; the
// waves of a block are independent. A strip overlaps its neighbours by the
// stages' combined x-radius (lanes near the strip edge compute values that
// only the neighbouring strip stores), and a chunk starts and ends the same
// number of rows early and late. Every load is a contiguous 64-node row.
//
// A smoothing sweep is written in the Jacobi form (see jacobi()), which
// needs only w/D and the real couplings, so its result can differ from the
// LDS-tiled kernels' residual form in the last bits.

#include "hz_device.h"

namespace hz {

namespace {

constexpr int kLanes = 64;

// Coefficients of the stencil of node_coef / stencil split by what they
// depend on: the column (fixed per lane) and the row (the same over the
// wavefront); only the shifted/absorbing term kap needs the node's slowness.
struct AxisC {
  double w, e, l;  // weight (1/2 at an end node), end nodes at the index (0..2), 2 - e
};
__device__ __forceinline__ AxisC axis_coef(int i, int n) {
  const int e = (i == 0) + (i == n - 1);
  AxisC a;
  a.w = e ? 0.5 : 1.0;
  a.e = (double)e;
  a.l = (double)(2 - e);
  return a;
}
// (M x)_p = (lsum x_p - wz sx - wx sz) / h^2 + kap x_p with lsum = wz lx + wx lz,
// kap = -omega^2 s wx wz m^2 + i omega g m / h and g = wz ex + wx ez;
// ka = -omega^2 Re s, kb = -omega^2 Im s, kc = omega / h
__device__ __forceinline__ double2 apply_m(const AxisC& cx, const AxisC& rz, double m, double ka, double kb,
                                           double kc, double ih2, double2 xp, double2 sx, double2 sz) {
  const double g = rz.w * cx.e + cx.w * rz.e;
  const double mw = (cx.w * rz.w) * (m * m);
  const double kre = ka * mw, kim = kb * mw + kc * g * m;
  const double lsum = rz.w * cx.l + cx.w * rz.l;
  const double lre = lsum * xp.x - rz.w * sx.x - cx.w * sz.x;
  const double lim = lsum * xp.y - rz.w * sx.y - cx.w * sz.y;
  return c2(ih2 * lre + (kre * xp.x - kim * xp.y), ih2 * lim + (kre * xp.y + kim * xp.x));
}
// One damped-Jacobi update u + (w/D)(b - M u) at a node, written as
// (1 - w) u + (w/D)(b + (wz sx + wx sz) / h^2): the couplings of M to the
// neighbours are real and its diagonal D (which holds the complex shift and
// the absorbing term) enters only through wd = w/D, so the slowness is not
// needed. cz = wz / h^2, cx = wx / h^2, omw = 1 - w.
__device__ __forceinline__ double2 jacobi(double2 u, double2 b, double2 wd, double2 sx, double2 sz, double cz,
                                          double cx, double omw) {
  const double tx = cz * sx.x + (cx * sz.x + b.x);
  const double ty = cz * sx.y + (cx * sz.y + b.y);
  return c2(omw * u.x + (wd.x * tx - wd.y * ty), omw * u.y + (wd.x * ty + wd.y * tx));
}


// One wave of a block: which (slot, strip, chunk) it owns. Blocks are mapped
// to XCDs as in decode_tile, over groups of four waves.
struct WaveTile {
  int slot, z0, z1, xs;
};

// chunk: rows per wave (even, so that coarse rows split evenly between waves)
__device__ __forceinline__ bool wave_tile(const Batch& bt, int nstrip, int nchunk, int chunk_rows, int groups,
                                          int width, int nz, WaveTile& w) {
  int slot, grp;
  if (!decode_tile(bt, groups, slot, grp)) return false;
  // the wavefront's index in the block, read from lane 0 so that the compiler
  // sees it (and every row index and row condition derived from it) as uniform
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kLanes));
  const int tile = grp * (kBlock / kLanes) + wv;
  if (tile >= nstrip * nchunk) return false;
  const int chunk = tile / nstrip, strip = tile - chunk * nstrip;
  w.slot = slot;
  w.z0 = chunk * chunk_rows;
  w.z1 = min(nz, w.z0 + chunk_rows);
  w.xs = strip * width;  // first column the strip stores
  return true;
}

}  // namespace

// The march is unrolled by two rows, and the loads of the next pair of rows
// are issued before the current pair is computed (software pipelining), so
// a wave keeps two pairs of rows in flight. Loads are unconditional, from
// row and column indices clamped into the grid; a value outside the grid is
// replaced by zero where it is used.

// Pre-smoothing and restriction (see launch_pre2r): per row j of the march,
// b_j and u1_j = (w/D) b_j are formed, u2 on row j-1 (one damped-Jacobi
// sweep from u1), the residual r = b - M u2 on row j-2, and, when row j-2 is
// odd, the full-weighting restriction to coarse row (j-3)/2 from r on rows
// j-4 .. j-2. x-radius 3 (u2, r, weights), z from z0-3 to z1+2. Lanes
// 3 .. 60 store: fine columns xs .. xs+57, coarse columns at even x. The
// pre-smoothed u2 is stored only when u2 is not null: the fused
// post-smoothing kernel forms it again from b (cheaper than writing and
// reading it back).
//
// MODE 4 and 5 form the operator product B p^ themselves instead of reading
// a stored v = B p^: p = r + beta (p_old - omega B p^_old) (p = r where beta
// is zero: the first iteration and the one after a restart, where p^_old
// holds nothing of this solve and its value is not used), and
// s = r - alpha B p^. B p^ on row j comes from p^ on
// rows j-1 .. j+1, loaded one row ahead of the other inputs; it widens the
// x-radius to 4, so those strips store 56 columns.
constexpr int pre_radius(int mode) { return mode >= 4 ? 4 : 3; }
constexpr int pre_width(int mode) { return kLanes - 2 * pre_radius(mode); }

template <int MODE>
struct PreRow {  // loads of one row: the right-hand side's inputs, w/D and m (MODE 4, 5: c is p^ on the next row)
  double2 a, b, c, wd;
  double m;
  double cr, cd, gb;  // with a density: the row's coupling table (RhoC)
};

// The couplings at lane x of row i from the row's own table entries (cr, cd)
// and the lower coupling of the row above (cd_up); every lane takes part in
// the lane shift.
__device__ __forceinline__ RhoC rho_row(int x, int i, double cr, double cd, double cd_up) {
  const double l = dpp_shift<kDppWaveShr1>(cr);
  RhoC c;
  c.l = x > 0 ? l : 0.0;
  c.r = cr;
  c.u = i > 0 ? cd_up : 0.0;
  c.d = cd;
  return c;
}

// FINE: launched on the finest level (the same code; a separate symbol lets a
// profiler tell the finest level's launches from the coarser ones). MODE 4
// and 5 hold p^ on three rows more: they get up to 168 VGPRs (3 waves per
// SIMD) rather than spill at 128, which made them far slower. RHO: with a
// density (Eq. (1)), the couplings come from the level's table (g.dc), kept
// for two rows behind the march; 3 waves per SIMD as well.
template <int MODE, bool FINE, bool RHO>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MODE >= 4 || RHO ? 3 : 4, 8))) k_pre2r_s(Grid g, Grid gc, int nstrip, int nchunk, int chunk_rows, int groups, int lvl,
                                                    Batch bt, RhsIn in, double2* __restrict__ bout,
                                                    double2* __restrict__ u2, double2* __restrict__ bc,
                                                    size_t stride, size_t sc) {
  constexpr int R = pre_radius(MODE), W = pre_width(MODE);
  WaveTile w;
  if (!wave_tile(bt, nstrip, nchunk, chunk_rows, groups, W, g.nz, w)) return;
  const int lane = threadIdx.x % kLanes;
  const Slot& S = bt.slots[w.slot];
  const FreqTab& f = bt.ft[S.freq];
  double2 beta = c2(0.0, 0.0), om = c2(0.0, 0.0), al = c2(0.0, 0.0);
  if (MODE == 1 || MODE == 4) {
    beta = S.beta;
    om = S.omega;
  }
  if (MODE == 2 || MODE == 5) al = S.alpha;
  const bool fresh = MODE == 4 && czero(beta);
  const int x = w.xs - R + lane;
  const bool xin = x >= 0 && x < g.nx;
  const int xx = min(max(x, 0), g.nx - 1);
  const bool own = lane >= R && lane < R + W && xin;
  const bool cown = own && !(x & 1);
  const size_t base = (size_t)w.slot * stride;
  const double2* wd = f.winv[lvl];
  const double ih = 1.0 / g.h, ih2 = ih * ih;
  const double om2 = f.omega * f.omega;
  const double ka = -om2 * f.sM_re, kb = -om2 * f.sM_im, kc = f.omega * ih;
  const double kaB = -om2 * f.sB_re, kbB = -om2 * f.sB_im;
  const double omw = 1.0 - f.wj[lvl];
  const AxisC cx = axis_coef(x, g.nx);
  const double cwx = ih2 * cx.w;
  const double2 zero = c2(0.0, 0.0);
  // node (j, xx) in the tables ([nz][nx]) and in the vectors (row pitch vp)
  const int vp = vpitch(g);
  auto row_index = [&](int j) { return (size_t)min(max(j, 0), g.nz - 1) * g.nx + xx; };
  auto vrow_index = [&](int j) { return (size_t)min(max(j, 0), g.nz - 1) * vp + xx; };
  const size_t nn = (size_t)g.nz * g.nx;
  auto load_row = [&](int j) {
    PreRow<MODE> r;
    const size_t q = row_index(j), qv = vrow_index(j);
    r.a = in.a[base + qv];
    if (MODE != 0 && MODE != 5) r.b = in.b[base + qv];
    if (MODE == 1) r.c = in.c[base + qv];
    if (MODE >= 4) r.c = in.c[base + vrow_index(j + 1)];
    r.wd = wd[q];
    r.m = model_m(g, f)[q];
    if (RHO) {
      r.cr = g.dc[q];
      r.cd = g.dc[nn + q];
      r.gb = g.dc[2 * nn + q];
    }
    return r;
  };
  // p^ on the rows of the grid, zero outside it (the operator's missing neighbours)
  auto p_hat = [&](int j, double2 v) { return keep(xin && j >= 0 && j < g.nz, v); };
  // weight of the right neighbour in the horizontal restriction stencil: 1
  // for the last fine node of an even-count axis (P^T of the clamped
  // interpolation), else 1/2
  const double wgx = x + 2 == g.nx ? 1.0 : 0.5;
  // rolling rows: u1 on j-2, j-1; b, m on j-1, j-2; w/D on j-1; u2 on j-3, j-2;
  // the horizontally restricted residual on j-4, j-3
  double2 u1a = zero, u1b = zero, b1 = zero, b2 = zero, wd1 = zero, u2a = zero, u2b = zero, ha = zero, hb = zero;
  double m1 = 0.0, m2 = 0.0;
  // RHO: the coupling table on rows j-1 and j-2, and the lower coupling of row j-3
  double cr1 = 0.0, cd1 = 0.0, gb1 = 0.0, cr2 = 0.0, cd2 = 0.0, gb2 = 0.0, cd3 = 0.0;
  // MODE 4, 5: p^ on rows j-1 and j
  double2 q0 = zero, q1 = zero;
  if (MODE >= 4) {
    q0 = p_hat(w.z0 - 4, in.c[base + vrow_index(w.z0 - 4)]);
    q1 = p_hat(w.z0 - 3, in.c[base + vrow_index(w.z0 - 3)]);
    // B p^ on the first row of the march couples to the row above it
    if (RHO) cd1 = g.dc[nn + row_index(w.z0 - 4)];
  }
  auto step = [&](int j, const PreRow<MODE>& L, bool odd) {
    const bool jin = xin && j >= 0 && j < g.nz;
    double2 bj = zero;
    if (MODE == 0) bj = L.a;
    if (MODE == 1) bj = cadd(L.a, cmul(beta, csub(L.b, cmul(om, L.c))));
    if (MODE == 2) bj = csub(L.a, cmul(al, L.b));
    if (MODE >= 4) {
      const double2 q2 = p_hat(j + 1, L.c);
      double2 bp;
      if (RHO) {
        const RhoC cj = rho_row(x, j, L.cr, L.cd, cd1);
        bp = apply_m_rho(cj, L.gb, cx.w * axis_coef(j, g.nz).w, L.m, kaB, kbB, kc, ih2, q1, from_left(q1),
                         from_right(q1), q0, q2);
      } else {
        bp = apply_m(cx, axis_coef(j, g.nz), L.m, kaB, kbB, kc, ih2, q1, cadd(from_left(q1), from_right(q1)),
                     cadd(q0, q2));
      }
      q0 = q1;
      q1 = q2;
      if (MODE == 4) bj = fresh ? L.a : cadd(L.a, cmul(beta, csub(L.b, cmul(om, bp))));
      if (MODE == 5) bj = csub(L.a, cmul(al, bp));
    }
    // outside the grid u1 = 0 through w/D; b and m there only enter values that are zeroed
    const double2 wdj = keep(jin, L.wd);
    const double mj = L.m;
    const double2 u1c = cmul(bj, wdj);
    // u2 on row j-1
    const int i2 = j - 1;
    double2 u2c = zero;
    {
      double2 v;
      if (RHO) {
        v = jacobi_rho(u1b, b1, wd1, rho_row(x, i2, cr1, cd1, cd2), from_left(u1b), from_right(u1b), u1a, u1c,
                       ih2, omw);
      } else {
        const double2 sx = cadd(from_left(u1b), from_right(u1b));
        const double2 sz = cadd(u1a, u1c);
        v = jacobi(u1b, b1, wd1, sx, sz, ih2 * axis_coef(i2, g.nz).w, cwx, omw);
      }
      u2c = keep(xin && i2 >= 0 && i2 < g.nz, v);
    }
    if (own && i2 >= w.z0 && i2 < w.z1) {
      const size_t q = base + (size_t)i2 * vp + x;
      if (MODE != 0) st_nt(bout + q, b1);
      if (u2) u2[q] = u2c;
    }
    // residual on row j-2
    const int ir = j - 2;
    double2 rc = zero;
    {
      double2 v;
      if (RHO) {
        const RhoC cir = rho_row(x, ir, cr2, cd2, cd3);
        v = csub(b2, apply_m_rho(cir, gb2, cx.w * axis_coef(ir, g.nz).w, m2, ka, kb, kc, ih2, u2b, from_left(u2b),
                                 from_right(u2b), u2a, u2c));
      } else {
        const double2 sx = cadd(from_left(u2b), from_right(u2b));
        const double2 sz = cadd(u2a, u2c);
        v = csub(b2, apply_m(cx, axis_coef(ir, g.nz), m2, ka, kb, kc, ih2, u2b, sx, sz));
      }
      rc = keep(xin && ir >= 0 && ir < g.nz, v);
    }
    // full weighting: each residual row restricted horizontally once, then
    // coarse row (ir - 1) / 2 from rows ir-2 .. ir (the last fine row of an
    // even-count axis again with weight 1)
    const double2 lc = from_left(rc), gc2 = from_right(rc);
    const double2 hc = c2(rc.x + 0.5 * lc.x + wgx * gc2.x, rc.y + 0.5 * lc.y + wgx * gc2.y);
    if (odd) {
      const int Iz = (ir - 1) / 2;
      if (cown && 2 * Iz >= w.z0 && 2 * Iz < w.z1 && Iz < gc.nz) {
        const double wz3 = 2 * Iz + 2 == g.nz ? 1.0 : 0.5;
        const double2 acc = c2(0.5 * ha.x + hb.x + wz3 * hc.x, 0.5 * ha.y + hb.y + wz3 * hc.y);
        bc[(size_t)w.slot * sc + (size_t)Iz * gc.nx + (x >> 1)] = cscale(0.25, acc);
      }
    }
    u1a = u1b;
    u1b = u1c;
    b2 = b1;
    b1 = bj;
    m2 = m1;
    m1 = mj;
    wd1 = wdj;
    u2a = u2b;
    u2b = u2c;
    ha = hb;
    hb = hc;
    if (RHO) {
      cd3 = cd2;
      cr2 = cr1;
      cd2 = cd1;
      gb2 = gb1;
      cr1 = L.cr;
      cd1 = L.cd;
      gb1 = L.gb;
    }
  };
  // rows z0-3 .. z1+2; the first row is odd (z0 even), so pairs are (odd, even)
  for (int j = w.z0 - 3; j <= w.z1 + 2; j += 2) {
    const PreRow<MODE> c0 = load_row(j), c1 = load_row(j + 1);
    step(j, c0, true);
    step(j + 1, c1, false);
  }
}

// Prolongation, correction and two post-sweeps (see launch_post2), with the
// pre-smoothed iterate formed again from b: per row j of the march,
// u1 = (w/D) b on row j, u2 (one sweep from u1, as in k_pre2r_s) and
// u3 = u2 + P e on row j-1, the first post-sweep u4 on row j-2, the second
// on row j-3, stored. x-radius 3, z from z0-3 to z1+2. Lanes 3 .. 60 store.
// HBM traffic per node: b and u_out, plus e on the coarse grid.
constexpr int kPostWidth = kLanes - 6;

struct PostRow {  // loads of one row j: b and w/D (with a density also row j-1's coupling table)
  double2 b, wd;
  double cr, cd;
};

// RHO: with a density (Eq. (1)), the couplings come from the level's table
// (g.dc), loaded one row behind b and kept for two rows; 3 waves per SIMD.
template <bool FINE, bool RHO>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RHO ? 3 : 4, 8))) k_post2_s(Grid gf, Grid gc, int nstrip, int nchunk, int chunk_rows, int groups, int lvl,
                                                    Batch bt, const double2* __restrict__ e,
                                                    const double2* __restrict__ b,
                                                    double2* __restrict__ u_out, size_t sf, size_t sc) {
  WaveTile w;
  if (!wave_tile(bt, nstrip, nchunk, chunk_rows, groups, kPostWidth, gf.nz, w)) return;
  const int lane = threadIdx.x % kLanes;
  const FreqTab& f = bt.ft[bt.slots[w.slot].freq];
  const int x = w.xs - 3 + lane;
  const bool xin = x >= 0 && x < gf.nx;
  const int xx = min(max(x, 0), gf.nx - 1);
  const bool own = lane >= 3 && lane < 3 + kPostWidth && xin;
  const size_t base = (size_t)w.slot * sf;
  const double2* es = e + (size_t)w.slot * sc;
  const double2* bs = b + base;
  const double2* wd = f.winv[lvl];
  const double ih = 1.0 / gf.h, ih2 = ih * ih;
  const double omw = 1.0 - f.wj[lvl];
  const double cwx = ih2 * axis_coef(x, gf.nx).w;
  const double2 zero = c2(0.0, 0.0);
  const int ox = x & 1;
  const int Jx = xx >> 1, Jx1 = min(Jx + 1, gc.nx - 1);
  const size_t nn = (size_t)gf.nz * gf.nx;
  const int vp = vpitch(gf);  // row pitch of b and u_out (the tables have nx)
  auto load_row = [&](int j) {
    PostRow r;
    const int jc = min(max(j, 0), gf.nz - 1);
    const size_t q = (size_t)jc * gf.nx + xx;
    r.b = bs[(size_t)jc * vp + xx];
    r.wd = wd[q];
    if (RHO) {
      const size_t q1 = (size_t)min(max(j - 1, 0), gf.nz - 1) * gf.nx + xx;
      r.cr = gf.dc[q1];
      r.cd = gf.dc[nn + q1];
    }
    return r;
  };
  auto load_coarse = [&](int cr, double2& ea, double2& eb) {
    const double2* row = es + (size_t)min(max(cr, 0), gc.nz - 1) * gc.nx;
    ea = row[Jx];
    eb = row[Jx1];
  };
  auto inside = [&](int j) { return xin && j >= 0 && j < gf.nz; };
  // rolling rows: u1 on j-2, j-1; u3 on j-3, j-2; u4 on j-4, j-3;
  // b, w/D on j-1, j-2, j-3
  double2 u1a = zero, u1b = zero, u3a = zero, u3b = zero, u4a = zero, u4b = zero;
  double2 b1 = zero, b2 = zero, b3 = zero, w1 = zero, w2 = zero, w3 = zero;
  // RHO: the coupling table on rows j-2 and j-3, and the lower coupling of row j-4
  double cr2 = 0.0, cd2 = 0.0, cr3 = 0.0, cd3 = 0.0, cd4 = 0.0;
  // lo, hi: coarse rows (j-1) >> 1 and the one below it
  auto step = [&](int j, const PostRow& L, double2 loa, double2 lob, double2 hia, double2 hib, bool odd_prev) {
    // outside the grid u1 = 0 through w/D; b there only enters values that are zeroed
    const double2 bj = L.b, wdj = keep(inside(j), L.wd);
    const double2 u1c = cmul(bj, wdj);
    // u2 and u3 on row j-1
    const int i2 = j - 1;
    double2 u3c;
    {
      double2 u2;
      if (RHO) {
        u2 = jacobi_rho(u1b, b1, w1, rho_row(x, i2, L.cr, L.cd, cd2), from_left(u1b), from_right(u1b), u1a, u1c,
                        ih2, omw);
      } else {
        const double2 sx = cadd(from_left(u1b), from_right(u1b));
        const double2 sz = cadd(u1a, u1c);
        u2 = jacobi(u1b, b1, w1, sx, sz, ih2 * axis_coef(i2, gf.nz).w, cwx, omw);
      }
      double2 a = ox ? cscale(0.5, cadd(loa, lob)) : loa;
      if (odd_prev) {
        const double2 a2 = ox ? cscale(0.5, cadd(hia, hib)) : hia;
        a = cscale(0.5, cadd(a, a2));
      }
      u3c = keep(inside(i2), cadd(u2, a));
    }
    // first post-sweep on row j-2
    const int i4 = j - 2;
    double2 u4c;
    if (RHO) {
      u4c = keep(inside(i4), jacobi_rho(u3b, b2, w2, rho_row(x, i4, cr2, cd2, cd3), from_left(u3b), from_right(u3b),
                                        u3a, u3c, ih2, omw));
    } else {
      const double2 sx = cadd(from_left(u3b), from_right(u3b));
      const double2 sz = cadd(u3a, u3c);
      u4c = keep(inside(i4), jacobi(u3b, b2, w2, sx, sz, ih2 * axis_coef(i4, gf.nz).w, cwx, omw));
    }
    // second post-sweep on row j-3
    const int i5 = j - 3;
    if (RHO) {
      const RhoC c5 = rho_row(x, i5, cr3, cd3, cd4);
      const double2 ul = from_left(u4b), ur = from_right(u4b);
      if (own && i5 >= w.z0 && i5 < w.z1)
        st_nt(u_out + base + (size_t)i5 * vp + x, jacobi_rho(u4b, b3, w3, c5, ul, ur, u4a, u4c, ih2, omw));
    } else {
      const double2 sx = cadd(from_left(u4b), from_right(u4b));
      if (own && i5 >= w.z0 && i5 < w.z1) {
        const double2 sz = cadd(u4a, u4c);
        st_nt(u_out + base + (size_t)i5 * vp + x, jacobi(u4b, b3, w3, sx, sz, ih2 * axis_coef(i5, gf.nz).w, cwx, omw));
      }
    }
    u1a = u1b;
    u1b = u1c;
    u3a = u3b;
    u3b = u3c;
    u4a = u4b;
    u4b = u4c;
    b3 = b2;
    b2 = b1;
    b1 = bj;
    w3 = w2;
    w2 = w1;
    w1 = wdj;
    if (RHO) {
      cd4 = cd3;
      cr3 = cr2;
      cd3 = cd2;
      cr2 = L.cr;
      cd2 = L.cd;
    }
  };
  // rows z0-3 .. z1+2 in pairs (odd j, even j+1): the step of row j forms u3
  // on row j-1 (even, coarse row (j-1)/2 only) and the step of j+1 on row j
  // (odd, coarse rows (j-1)/2 and (j+1)/2)
  double2 loa, lob;
  load_coarse((w.z0 - 4) >> 1, loa, lob);
  for (int j = w.z0 - 3; j <= w.z1 + 2; j += 2) {
    double2 hia, hib;
    load_coarse((j + 1) >> 1, hia, hib);
    const PostRow c0 = load_row(j), c1 = load_row(j + 1);
    // row j-1 is even: its coarse row is (j-1)/2, held in lo
    step(j, c0, loa, lob, loa, lob, false);
    step(j + 1, c1, loa, lob, hia, hib, true);
    loa = hia;
    lob = hib;
  }
}

// ---------------------------------------------------------------- launchers
namespace {
struct StreamShape {
  int nstrip, nchunk, groups;
};
StreamShape stream_shape(const Grid& g, int width, int chunk_rows) {
  StreamShape s;
  s.nstrip = (g.nx + width - 1) / width;
  s.nchunk = (g.nz + chunk_rows - 1) / chunk_rows;
  s.groups = (s.nstrip * s.nchunk + (kBlock / kLanes) - 1) / (kBlock / kLanes);
  return s;
}
}  // namespace

hipError_t launch_pre2r(const Grid& g, const Grid& gc, int lvl, int mode, const Batch& bt, int cap,
                        const double2* a, const double2* b, const double2* c, double2* bout, double2* u2,
                        double2* bcoarse, size_t stride, size_t sc, int chunk_rows, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (chunk_rows < 2 || (chunk_rows & 1)) return hipErrorInvalidValue;
  if (g.rho && !g.dc) return hipErrorInvalidValue;  // a density needs the level's coupling table
  // modes other than 0 form the finest level's right-hand side
  if (mode < 0 || mode > 5 || mode == 3 || (lvl != 0 && mode != 0)) return hipErrorInvalidValue;
  const StreamShape sh = stream_shape(g, pre_width(mode), chunk_rows);
  const RhsIn in{a, b, c};
  const dim3 gr((unsigned)tile_blocks(sh.groups, cap));
#define HZ_PRE2R(M, F)                                                                                           \
  do {                                                                                                           \
    if (g.dc)                                                                                                    \
      hipLaunchKernelGGL((k_pre2r_s<M, F, true>), gr, dim3(kBlock), 0, st, g, gc, sh.nstrip, sh.nchunk,         \
                         chunk_rows, sh.groups, lvl, bt, in, bout, u2, bcoarse, stride, sc);                     \
    else                                                                                                         \
      hipLaunchKernelGGL((k_pre2r_s<M, F, false>), gr, dim3(kBlock), 0, st, g, gc, sh.nstrip, sh.nchunk,        \
                         chunk_rows, sh.groups, lvl, bt, in, bout, u2, bcoarse, stride, sc);                     \
  } while (0)
  if (mode == 1) HZ_PRE2R(1, true);
  else if (mode == 2) HZ_PRE2R(2, true);
  else if (mode == 4) HZ_PRE2R(4, true);
  else if (mode == 5) HZ_PRE2R(5, true);
  else if (lvl == 0) HZ_PRE2R(0, true);
  else HZ_PRE2R(0, false);
#undef HZ_PRE2R
  return hipGetLastError();
}

hipError_t launch_post2(const Grid& gf, const Grid& gc, int lvl, const Batch& bt, int cap, const double2* e,
                        const double2* b, double2* u_out, size_t sf, size_t sc, int chunk_rows, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (chunk_rows < 2 || (chunk_rows & 1)) return hipErrorInvalidValue;
  if (gf.rho && !gf.dc) return hipErrorInvalidValue;  // a density needs the level's coupling table
  const StreamShape sh = stream_shape(gf, kPostWidth, chunk_rows);
  const dim3 gr((unsigned)tile_blocks(sh.groups, cap));
#define HZ_POST2(F, R)                                                                                          \
  hipLaunchKernelGGL((k_post2_s<F, R>), gr, dim3(kBlock), 0, st, gf, gc, sh.nstrip, sh.nchunk, chunk_rows,   \
                     sh.groups, lvl, bt, e, b, u_out, sf, sc)
  if (gf.dc) {
    if (lvl == 0) HZ_POST2(true, true);
    else HZ_POST2(false, true);
  } else {
    if (lvl == 0) HZ_POST2(true, false);
    else HZ_POST2(false, false);
  }
#undef HZ_POST2
  return hipGetLastError();
}

}  // namespace hz
