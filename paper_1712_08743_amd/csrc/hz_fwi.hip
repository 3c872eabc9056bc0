// HIP kernels of the FWI gradient (gfx950): adjoint sources from the data
// residual, and the adjoint-state accumulation of dJ/dm.
//
// Eq. (4): J(m) = sum |u_obs - u_cal(m)|^2 + lambda sum m^2 (shots, receivers,
// frequencies). Eq. (7) gives its gradient through the Frechet derivative;
// with res = P u - d_obs and the adjoint field mu solving B mu = P^T conj(res)
// (B is complex symmetric, so the transpose system is B itself),
//   dJ/dm_i = -2 Re[ sum_{f,s} delta_i(f) u_i mu_i ] + 2 lambda m_i,
//   delta_i(f) = dB_ii/dm_i = j omega g_i / h - 2 omega^2 (1 - j alpha) w_i m_i,
// the absorbing boundary term included; on 1D, 2D and 3D grids (g_i the
// node's exposed boundary length or face area, w_i its control volume).

#include "hz_device.h"
#include "hz_node3.h"

namespace hz {

// out[slot] = P^T conj(P u - d_obs) for every slot: zero everywhere except at
// receiver nodes. Receivers sharing a node are summed in receiver order
// (rec_ptr / rec_idx list the receivers of each distinct node).
__global__ void k_adjoint_zero(size_t total, double2* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = c2(0.0, 0.0);
}

__global__ void k_adjoint_set(int nslots, int nuniq, const int* __restrict__ uniq_node,
                              const int* __restrict__ rec_ptr, const int* __restrict__ rec_idx,
                              int nrec, const double2* __restrict__ u,
                              const double2* __restrict__ d_obs, double2* __restrict__ out,
                              size_t stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots * nuniq) return;
  const int s = i / nuniq, k = i - s * nuniq;
  const int node = uniq_node[k];
  const double2 us = u[(size_t)s * stride + node];
  double2 acc = c2(0.0, 0.0);
  for (int q = rec_ptr[k]; q < rec_ptr[k + 1]; ++q) {
    const double2 r = csub(us, d_obs[(size_t)s * nrec + rec_idx[q]]);
    acc = cadd(acc, c2(r.x, -r.y));
  }
  out[(size_t)s * stride + node] = acc;
}

// The geometry of dB_ii/dm_i at node p: gh = g_i / h (the boundary term's
// weight over h) and w = w_i (the control-volume weight), on a 1D, 2D or 3D
// grid (flat index p).
template <int DIM>
__device__ __forceinline__ void sens_geom(const Grid& g, size_t p, double& gh, double& w) {
  if constexpr (DIM == 3) {
    const size_t r = p / g.nx;
    const int ix = (int)(p - r * g.nx), iz = (int)(r / g.ny), iy = (int)(r - (size_t)iz * g.ny);
    // with omega = m = 1 and no mass shift, kap.y is the boundary weight over h
    // (a density of Eq. (1) scales it by sqrt(rho_i))
    gh = node_coef3(iz, iy, ix, g, 1.0 / g.h, 1.0, 1.0, 0.0, 0.0).kap.y;
    if (g.rho) gh *= sqrt(g.rho[p]);
    w = (iz == 0 || iz == g.nz - 1 ? 0.5 : 1.0) * (iy == 0 || iy == g.ny - 1 ? 0.5 : 1.0) *
        (ix == 0 || ix == g.nx - 1 ? 0.5 : 1.0);
  } else {
    const int iz = DIM == 2 ? (int)(p / g.nx) : 0;
    const int ix = (int)(p - (size_t)iz * g.nx);
    // geometry weights: d(kap)/dm with s = 1 - j alpha and omega = 1 gives the per-frequency pieces
    const NodeC c1 = node_coef<DIM == 2>(iz, ix, g.nz, g.nx, 1.0 / g.h, 1.0, 1.0, 0.0, 0.0);  // kap.y = g / h
    // a density of Eq. (1) scales the absorbing term by sqrt(rho_i)
    gh = g.rho ? c1.kap.y * sqrt(g.rho[p]) : c1.kap.y;
    w = c1.wx * c1.wz;
  }
}

// grad_i = -2 Re sum_{f, s} delta_i(f) u_i mu_i + 2 lambda m_i, one thread per
// node, slots summed in order (deterministic). u and mu are [nfreq*nsrc][n].
// accumulate != 0 adds to grad (frequency chunks).
// The same sum serves the Gauss-Newton product H v = 2 Re[G^H G v] + 2 lambda v
// when mu is the adjoint field of the Born data of v: reg is m (gradient) or
// v (Gauss-Newton product).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_grad_accum(Grid g, int nfreq, int nsrc,
                                                       const double* __restrict__ omega, double alpha,
                                                       const double2* __restrict__ u,
                                                       const double2* __restrict__ mu, size_t stride,
                                                       double lambda, const double* __restrict__ reg,
                                                       int accumulate, double* __restrict__ grad) {
  const size_t n = (size_t)g.nz * g.ny * g.nx;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double m = g.m[p];
  double gh, w;
  sens_geom<DIM>(g, p, gh, w);
  double acc = 0.0;
  for (int f = 0; f < nfreq; ++f) {
    const double om = omega[f];
    // delta = j om g/h - 2 om^2 (1 - j alpha) w m
    const double t = 2.0 * om * om * w * m;
    const double2 delta = c2(-t, om * gh + t * alpha);
    double2 s = c2(0.0, 0.0);
    for (int k = 0; k < nsrc; ++k) {
      const size_t q = (size_t)(f * nsrc + k) * stride + p;
      s = cadd(s, cmul(u[q], mu[q]));
    }
    acc += cmul(delta, s).x;
  }
  const double val = -2.0 * acc;
  grad[p] = accumulate ? grad[p] + val : val + 2.0 * lambda * reg[p];
}

// Born right-hand sides: rhs[slot] = -delta(f) * u[slot] * v (v real).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_born_src(Grid g, int nslots, int nsrc,
                                                     const double* __restrict__ omega, double alpha,
                                                     const double2* __restrict__ u,
                                                     const double* __restrict__ v,
                                                     double2* __restrict__ rhs, size_t stride) {
  const size_t n = (size_t)g.nz * g.ny * g.nx;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double m = g.m[p];
  double gh, w;
  sens_geom<DIM>(g, p, gh, w);
  const double vp = v[p];
  for (int s = 0; s < nslots; ++s) {
    const double om = omega[s / nsrc];
    const double t = 2.0 * om * om * w * m;
    const double2 delta = c2(-t, om * gh + t * alpha);
    const size_t q = (size_t)s * stride + p;
    rhs[q] = cscale(-vp, cmul(delta, u[q]));
  }
}

// Adjoint right-hand sides of given receiver data y[slot][rec]:
// rhs[slot] = P^T conj(y), receivers sharing a node summed in receiver order.
__global__ void k_adjoint_data(int nslots, int nuniq, const int* __restrict__ uniq_node,
                               const int* __restrict__ rec_ptr, const int* __restrict__ rec_idx, int nrec,
                               const double2* __restrict__ y, double2* __restrict__ out, size_t stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots * nuniq) return;
  const int s = i / nuniq, k = i - s * nuniq;
  double2 acc = c2(0.0, 0.0);
  for (int q = rec_ptr[k]; q < rec_ptr[k + 1]; ++q) {
    const double2 r = y[(size_t)s * nrec + rec_idx[q]];
    acc = cadd(acc, c2(r.x, -r.y));
  }
  out[(size_t)s * stride + uniq_node[k]] = acc;
}

// Conjugate gradients on the Gauss-Newton system H dm = -g, one block
// (fixed-order sums). st[0] = r.r, st[1] = g.g, st[2] = done flag.
//   mode 0: x = 0, r = p = -g, r.r
//   mode 1: (Hp given) a = r.r / p.Hp, x += a p, r -= a Hp, p = r + (r.r'/r.r) p
__device__ __forceinline__ double block_dot_1024(double v) {
  __shared__ double sh[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  return t;  // every thread holds the sum
}

__global__ void __launch_bounds__(1024) k_cg(int mode, size_t n, const double* __restrict__ g,
                                             const double* __restrict__ Hp, double* __restrict__ x,
                                             double* __restrict__ r, double* __restrict__ p,
                                             double* __restrict__ st, double tol) {
  if (mode == 0) {
    double a = 0.0;
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
      const double ri = -g[i];
      x[i] = 0.0;
      r[i] = ri;
      p[i] = ri;
      a += ri * ri;
    }
    const double rr = block_dot_1024(a);
    if (threadIdx.x == 0) {
      st[0] = rr;
      st[1] = rr;
      st[2] = (rr == 0.0) ? 1.0 : 0.0;
    }
    return;
  }
  double a = 0.0;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) a += p[i] * Hp[i];
  const double pHp = block_dot_1024(a);
  const double rr = st[0];
  const double alpha = rr / pHp;
  double b = 0.0;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * Hp[i];
    r[i] = ri;
    b += ri * ri;
  }
  const double rr_new = block_dot_1024(b);
  const double beta = rr_new / rr;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = r[i] + beta * p[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    st[0] = rr_new;
    st[2] = (!(pHp > 0.0) || !isfinite(rr_new) || rr_new <= tol * tol * st[1]) ? 1.0 : 0.0;
  }
}

static inline unsigned flat_blocks(size_t total) {
  size_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return (unsigned)b;
}

hipError_t launch_adjoint_src(int nslots, size_t n, int nuniq, const int* uniq_node, const int* rec_ptr,
                              const int* rec_idx, int nrec, const double2* u, const double2* d_obs,
                              double2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_zero, dim3(flat_blocks(n * nslots)), dim3(256), 0, st, n * nslots, out);
  const int tot = nslots * nuniq;
  if (tot > 0)
    hipLaunchKernelGGL(k_adjoint_set, dim3((tot + 255) / 256), dim3(256), 0, st, nslots, nuniq, uniq_node,
                       rec_ptr, rec_idx, nrec, u, d_obs, out, n);
  return hipGetLastError();
}

hipError_t launch_grad_accum(int dim, const Grid& g, int nfreq, int nsrc, const double* omega, double alpha,
                             const double2* u, const double2* mu, double lambda, const double* reg,
                             int accumulate, double* grad, hipStream_t st) {
  const size_t n = (size_t)g.nz * g.ny * g.nx;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (dim == 3)
    hipLaunchKernelGGL(k_grad_accum<3>, dim3(nb), dim3(kBlock), 0, st, g, nfreq, nsrc, omega, alpha, u, mu, n,
                       lambda, reg, accumulate, grad);
  else if (dim == 2)
    hipLaunchKernelGGL(k_grad_accum<2>, dim3(nb), dim3(kBlock), 0, st, g, nfreq, nsrc, omega, alpha, u, mu, n,
                       lambda, reg, accumulate, grad);
  else
    hipLaunchKernelGGL(k_grad_accum<1>, dim3(nb), dim3(kBlock), 0, st, g, nfreq, nsrc, omega, alpha, u, mu, n,
                       lambda, reg, accumulate, grad);
  return hipGetLastError();
}

hipError_t launch_born_src(int dim, const Grid& g, int nslots, int nsrc, const double* omega, double alpha,
                           const double2* u, const double* v, double2* rhs, hipStream_t st) {
  const size_t n = (size_t)g.nz * g.ny * g.nx;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (dim == 3)
    hipLaunchKernelGGL(k_born_src<3>, dim3(nb), dim3(kBlock), 0, st, g, nslots, nsrc, omega, alpha, u, v, rhs, n);
  else if (dim == 2)
    hipLaunchKernelGGL(k_born_src<2>, dim3(nb), dim3(kBlock), 0, st, g, nslots, nsrc, omega, alpha, u, v, rhs, n);
  else
    hipLaunchKernelGGL(k_born_src<1>, dim3(nb), dim3(kBlock), 0, st, g, nslots, nsrc, omega, alpha, u, v, rhs, n);
  return hipGetLastError();
}

hipError_t launch_adjoint_data(int nslots, size_t n, int nuniq, const int* uniq_node, const int* rec_ptr,
                               const int* rec_idx, int nrec, const double2* y, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_zero, dim3(flat_blocks(n * nslots)), dim3(256), 0, st, n * nslots, out);
  const int tot = nslots * nuniq;
  if (tot > 0)
    hipLaunchKernelGGL(k_adjoint_data, dim3((tot + 255) / 256), dim3(256), 0, st, nslots, nuniq, uniq_node,
                       rec_ptr, rec_idx, nrec, y, out, n);
  return hipGetLastError();
}

hipError_t launch_cg(int mode, size_t n, const double* g, const double* Hp, double* x, double* r, double* p,
                     double* state, double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_cg, dim3(1), dim3(1024), 0, st, mode, n, g, Hp, x, r, p, state, tol);
  return hipGetLastError();
}

}  // namespace hz
