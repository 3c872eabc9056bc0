// The operator at a node of a 3D grid (Eq. (1) with d = 3, constant density
// as in Eq. (2)): nodes (iz, iy, ix), flat index (iz * ny + iy) * nx + ix,
// every face of the box absorbing. As in 1D and 2D, each row is the
// control-volume form: two neighbours along an axis are coupled by the face
// between their volumes, the product of the other two axes' end weights
// (1/2 at an end node, else 1); the boundary term carries the exposed face
// area; the mass term the volume, the product of all three weights.
//
// The 3D kernels tile the grid as a 2D one of nz * ny rows by nx columns
// (tile_node<true> over grid_tiles(nz * ny, nx, 3)), so the flat index and
// the reduction tiles are those of a 2D grid of that shape.
#pragma once

#include "hz_device.h"

namespace hz {

struct NodeC3 {
  double fz, fy, fx;  // couplings along z, y, x: the face weights
  double lsum;        // sum of the couplings to the existing neighbours
  double2 kap;        // boundary and mass term (diagonal part without lsum / h^2)
};

__device__ __forceinline__ NodeC3 node_coef3(int iz, int iy, int ix, const Grid& g, double ih, double m,
                                             double omega, double s_re, double s_im) {
  const int ez = (iz == 0) + (iz == g.nz - 1), ey = (iy == 0) + (iy == g.ny - 1), ex = (ix == 0) + (ix == g.nx - 1);
  const double wz = ez ? 0.5 : 1.0, wy = ey ? 0.5 : 1.0, wx = ex ? 0.5 : 1.0;
  NodeC3 c;
  c.fz = wy * wx;
  c.fy = wz * wx;
  c.fx = wz * wy;
  c.lsum = c.fz * (double)(2 - ez) + c.fy * (double)(2 - ey) + c.fx * (double)(2 - ex);
  const double gb = c.fz * (double)ez + c.fy * (double)ey + c.fx * (double)ex;
  const double om2wm2 = omega * omega * (wz * wy * wx) * (m * m);
  c.kap = c2(-om2wm2 * s_re, omega * gb * m * ih - om2wm2 * s_im);
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

// The node of a thread in the row-tiled 3D grid: false past the grid.
__device__ __forceinline__ bool node3_of(const Tiles& t, int tile, const Grid& g, int& iz, int& iy, int& ix,
                                         size_t& p) {
  int r;
  tile_node<true>(t, tile, r, ix);
  if (r >= g.nz * g.ny || ix >= g.nx) return false;
  iz = r / g.ny;
  iy = r - iz * g.ny;
  p = (size_t)r * g.nx + ix;
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
