// The operator at a node of a 3D grid (Eq. (1) with d = 3, constant density
// as in Eq. (2)): nodes (iz, iy, ix), flat index (iz * ny + iy) * nx + ix,
// every face of the box absorbing. As in 1D and 2D, each row is the
// control-volume form: two neighbours along an axis are coupled by the face
// between their volumes, the product of the other two axes' end weights
// (1/2 at an end node, else 1); the boundary term carries the exposed face
// area; the mass term the volume, the product of all three weights.
//
// The one-node-per-thread 3D kernels take kBlock consecutive nodes of the
// flat index per tile (node3_of over grid_tiles(nz * ny, nx, 3)); the
// reduction tiles are those tiles.
#pragma once

#include "hz_device.h"

namespace hz {

struct NodeC3 {
  double fz, fy, fx;  // couplings along z, y, x: the face weights
  double lsum;        // sum of the couplings to the existing neighbours
  double2 kap;        // boundary and mass term (diagonal part without lsum / h^2)
};

// gs scales the absorbing term (sqrt of the node's density, see node_op3)
__device__ __forceinline__ NodeC3 node_coef3(int iz, int iy, int ix, const Grid& g, double ih, double m,
                                             double omega, double s_re, double s_im, double gs = 1.0) {
  const int ez = (iz == 0) + (iz == g.nz - 1), ey = (iy == 0) + (iy == g.ny - 1), ex = (ix == 0) + (ix == g.nx - 1);
  const double wz = ez ? 0.5 : 1.0, wy = ey ? 0.5 : 1.0, wx = ex ? 0.5 : 1.0;
  NodeC3 c;
  c.fz = wy * wx;
  c.fy = wz * wx;
  c.fx = wz * wy;
  c.lsum = c.fz * (double)(2 - ez) + c.fy * (double)(2 - ey) + c.fx * (double)(2 - ex);
  const double gb = c.fz * (double)ez + c.fy * (double)ey + c.fx * (double)ex;
  const double om2wm2 = omega * omega * (wz * wy * wx) * (m * m);
  c.kap = c2(-om2wm2 * s_re, omega * gb * m * ih * gs - om2wm2 * s_im);
  return c;
}

__device__ __forceinline__ double2 diag3(const NodeC3& c, double ih2) { return c2(c.lsum * ih2 + c.kap.x, c.kap.y); }

// (A x)_p from x_p and the sums of its existing neighbours along each axis
__device__ __forceinline__ double2 stencil3(const NodeC3& c, double ih2, double2 xp, double2 sz, double2 sy,
                                            double2 sx) {
  const double2 lx = c2(c.lsum * xp.x - c.fz * sz.x - c.fy * sy.x - c.fx * sx.x,
                        c.lsum * xp.y - c.fz * sz.y - c.fy * sy.y - c.fx * sx.y);
  return cadd(cscale(ih2, lx), cmul(c.kap, xp));
}

// (A x)_p for x at the slot's base pointer, p the node's flat index. A
// neighbour past the grid is read at p itself and dropped, so the seven loads
// carry no branches and are issued together.
__device__ __forceinline__ double2 apply_node3(const double2* __restrict__ x, size_t p, int iz, int iy, int ix,
                                               const Grid& g, double ih2, const NodeC3& c) {
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const bool xl = ix > 0, xr = ix < g.nx - 1, yl = iy > 0, yr = iy < g.ny - 1, zl = iz > 0, zr = iz < g.nz - 1;
  const double2 vxl = x[xl ? p - 1 : p], vxr = x[xr ? p + 1 : p];
  const double2 vyl = x[yl ? p - sy : p], vyr = x[yr ? p + sy : p];
  const double2 vzl = x[zl ? p - sz : p], vzr = x[zr ? p + sz : p];
  const double2 zero = c2(0.0, 0.0);
  const double2 ax = cadd(cadd(zero, xl ? vxl : zero), xr ? vxr : zero);
  const double2 ay = cadd(cadd(zero, yl ? vyl : zero), yr ? vyr : zero);
  const double2 az = cadd(cadd(zero, zl ? vzl : zero), zr ? vzr : zero);
  return stencil3(c, ih2, x[p], az, ay, ax);
}

// ---- variable density (Eq. (1) with d = 3): the coupling to a neighbour is
// the face weight times the mean density of the two nodes, the absorbing
// term carries sqrt(rho_p) (as node_op in 2D). Grid::rho null: node_op3 and
// apply_op3 are node_coef3 and apply_node3.
struct NodeOp3 {
  NodeC3 c;      // lsum: the sum of the couplings in use
  double cq[6];  // density couplings to the -x, +x, -y, +y, -z, +z neighbours (0 where missing)
};

__device__ __forceinline__ NodeOp3 node_op3(int iz, int iy, int ix, const Grid& g, size_t p, double m, double omega,
                                            double s_re, double s_im) {
  NodeOp3 o;
  if (!g.rho) {
    o.c = node_coef3(iz, iy, ix, g, 1.0 / g.h, m, omega, s_re, s_im);
    return o;
  }
  const double* r = g.rho;
  const double rp = r[p];
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  o.c = node_coef3(iz, iy, ix, g, 1.0 / g.h, m, omega, s_re, s_im, sqrt(rp));
  o.cq[0] = ix > 0 ? o.c.fx * (0.5 * (rp + r[p - 1])) : 0.0;
  o.cq[1] = ix < g.nx - 1 ? o.c.fx * (0.5 * (rp + r[p + 1])) : 0.0;
  o.cq[2] = iy > 0 ? o.c.fy * (0.5 * (rp + r[p - sy])) : 0.0;
  o.cq[3] = iy < g.ny - 1 ? o.c.fy * (0.5 * (rp + r[p + sy])) : 0.0;
  o.cq[4] = iz > 0 ? o.c.fz * (0.5 * (rp + r[p - sz])) : 0.0;
  o.cq[5] = iz < g.nz - 1 ? o.c.fz * (0.5 * (rp + r[p + sz])) : 0.0;
  o.c.lsum = ((o.cq[0] + o.cq[1]) + (o.cq[2] + o.cq[3])) + (o.cq[4] + o.cq[5]);
  return o;
}

// (A x)_p with the value at p and the neighbours' values from val(dz, dy, dx),
// called for the existing neighbours only
template <class F>
__device__ __forceinline__ double2 apply_op3_at(const Grid& g, const NodeOp3& o, int iz, int iy, int ix, double ih2,
                                                double2 xp, F val) {
  if (!g.rho) {
    double2 sz = c2(0.0, 0.0), sy = c2(0.0, 0.0), sx = c2(0.0, 0.0);
    if (ix > 0) sx = cadd(sx, val(0, 0, -1));
    if (ix < g.nx - 1) sx = cadd(sx, val(0, 0, 1));
    if (iy > 0) sy = cadd(sy, val(0, -1, 0));
    if (iy < g.ny - 1) sy = cadd(sy, val(0, 1, 0));
    if (iz > 0) sz = cadd(sz, val(-1, 0, 0));
    if (iz < g.nz - 1) sz = cadd(sz, val(1, 0, 0));
    return stencil3(o.c, ih2, xp, sz, sy, sx);
  }
  double2 s = c2(0.0, 0.0);
  if (ix > 0) s = cadd(s, cscale(o.cq[0], val(0, 0, -1)));
  if (ix < g.nx - 1) s = cadd(s, cscale(o.cq[1], val(0, 0, 1)));
  if (iy > 0) s = cadd(s, cscale(o.cq[2], val(0, -1, 0)));
  if (iy < g.ny - 1) s = cadd(s, cscale(o.cq[3], val(0, 1, 0)));
  if (iz > 0) s = cadd(s, cscale(o.cq[4], val(-1, 0, 0)));
  if (iz < g.nz - 1) s = cadd(s, cscale(o.cq[5], val(1, 0, 0)));
  const double2 lx = c2(o.c.lsum * xp.x - s.x, o.c.lsum * xp.y - s.y);
  return cadd(cscale(ih2, lx), cmul(o.c.kap, xp));
}

// (A x)_p for x at the slot's base pointer
__device__ __forceinline__ double2 apply_op3(const Grid& g, const NodeOp3& o, const double2* __restrict__ x, size_t p,
                                             int iz, int iy, int ix, double ih2) {
  if (!g.rho) return apply_node3(x, p, iz, iy, ix, g, ih2, o.c);
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  return apply_op3_at(g, o, iz, iy, ix, ih2, x[p], [&](int dz, int dy, int dx) {
    return x[(size_t)((long long)p + (long long)dz * (long long)sz + (long long)dy * (long long)sy + dx)];
  });
}

// The node of a thread: node tile * kBlock + thread of the flat index
// (iz * ny + iy) * nx + ix; false past the grid. (Rows of 129 nodes tiled
// 64 columns wide left a third of the threads idle.)
__device__ __forceinline__ bool node3_of(const Tiles& t, int tile, const Grid& g, int& iz, int& iy, int& ix,
                                         size_t& p) {
  (void)t;
  const size_t q = (size_t)tile * kBlock + threadIdx.x;
  if (q >= (size_t)g.nz * g.ny * g.nx) return false;
  const int r = (int)(q / (size_t)g.nx);
  ix = (int)(q - (size_t)r * g.nx);
  iz = r / g.ny;
  iy = r - iz * g.ny;
  p = q;
  return true;
}

// Trilinear interpolation of coarse e (nc axes) at fine node (iz, iy, ix): the
// tensor product of the axes' linear interpolations. The last node of an
// even-count axis has no upper coarse neighbour: the clamped index makes its
// average (e_J + e_J) / 2 = e_J exactly.
__device__ __forceinline__ double2 interp3(const double2* __restrict__ e, int iz, int iy, int ix, int ncz, int ncy,
                                           int ncx) {
  const int Jx = ix >> 1, ox = ix & 1, Jx1 = min(Jx + 1, ncx - 1);
  const int Jy = iy >> 1, oy = iy & 1, Jy1 = min(Jy + 1, ncy - 1);
  const int Jz = iz >> 1, oz = iz & 1, Jz1 = min(Jz + 1, ncz - 1);
  auto line = [&](int jz, int jy) {
    const double2* r = e + ((size_t)jz * ncy + jy) * ncx;
    return ox ? cscale(0.5, cadd(r[Jx], r[Jx1])) : r[Jx];
  };
  auto plane = [&](int jz) { return oy ? cscale(0.5, cadd(line(jz, Jy), line(jz, Jy1))) : line(jz, Jy); };
  return oz ? cscale(0.5, cadd(plane(Jz), plane(Jz1))) : plane(Jz);
}

}  // namespace hz
