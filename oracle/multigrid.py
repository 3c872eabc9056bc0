"""ORACLE (test infrastructure only): geometric V-cycle approximating M^-1.

The paper preconditions its Krylov data-modelling engine with the
shifted-Laplace operator M = -Laplace - (beta1 - j beta2) omega^2 m^2 (section
on FWI, where the GMRES engine is preconditioned; Examples: complex shift
"1 + j"). It does not say how M^-1 is applied. The method applied here is one
geometric multigrid V-cycle, written out plainly:

* levels l = 0..L-1, grid n_l = (n - 1) / 2^l + 1 per axis, spacing 2^l h;
* the slowness on level l is m injected at the coincident nodes, and M_l is
  rediscretised there with the same formula as the fine operator;
* damped Jacobi smoothing u <- u + w_l (b - M_l u) / diag(M_l), nu1 sweeps
  before and nu2 after the coarse correction, starting from u = 0;
* restriction R = 2^-dim P^T of the weighted residual (full weighting in the
  interior), bilinear prolongation P (linear in 1D, trilinear in 3D);
* exact solve on the coarsest level (SuperLU here; any exact method is the
  same operator).

With L = 1 the V-cycle is the exact solve of M on the fine grid.
"""

import numpy as np
import scipy.sparse as sp

from .operator import operator_M
from .direct import factor_superlu


def coarse_size(n):
    """Nodes of the next coarser grid along an axis: coarse node J sits on
    fine node 2J. With an odd node count the two grids share both ends; with
    an even count the last fine node has no coarse partner and is
    interpolated from the last coarse node alone (the coarse grid then ends
    one fine spacing short of the fine boundary)."""
    return (n + 1) // 2


def coarse_shape(shape):
    """Shape of the next coarser grid; raises if an axis would drop below
    three nodes."""
    out = []
    for n in shape:
        if n < 5:
            raise ValueError(f"grid axis {n} cannot be coarsened")
        out.append(coarse_size(n))
    return tuple(out)


def inject(m):
    """Slowness on the next coarser grid: values at the coincident nodes."""
    m = np.asarray(m)
    return m[(slice(None, None, 2),) * m.ndim]


def linear_interp_1d(nc, nf=None):
    """nf x nc linear interpolation: copy at even fine nodes, average of the
    two neighbours at odd ones; an odd fine node with no right coarse
    neighbour (the last node of an even count) copies the last coarse value."""
    if nf is None:
        nf = 2 * (nc - 1) + 1
    if nf not in (2 * nc - 1, 2 * nc):
        raise ValueError("fine axis must have 2 nc - 1 or 2 nc nodes")
    rows, cols, vals = [], [], []
    for i in range(nf):
        I = i // 2
        if i % 2 == 0:
            rows.append(i), cols.append(I), vals.append(1.0)
        elif I + 1 < nc:
            rows += [i, i]
            cols += [I, I + 1]
            vals += [0.5, 0.5]
        else:
            rows.append(i), cols.append(I), vals.append(1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def prolongation(coarse, fine=None):
    """Linear (1D), bilinear (2D) or trilinear (3D) prolongation from a coarse
    grid shape to the fine shape (default: the odd-count fine grid 2 nc - 1):
    the tensor product of the axes' linear interpolations."""
    if fine is None:
        fine = tuple(2 * (n - 1) + 1 for n in coarse)
    P = linear_interp_1d(coarse[0], fine[0])
    # flat order: the first axis is the slow (outer) factor of the Kronecker product
    for a in range(1, len(coarse)):
        P = sp.kron(P, linear_interp_1d(coarse[a], fine[a]))
    return P.tocsr()


def restriction(coarse, fine=None):
    """R = 2^-dim P^T (full weighting in the interior)."""
    return (prolongation(coarse, fine).T * (0.5 ** len(coarse))).tocsr()


class VCycle:
    """One V-cycle V(nu1, nu2) as a fixed linear map b -> u ~ M^-1 b.

    wj: one damped-Jacobi weight per smoothing level (levels 0..L-2).
    coarse: "exact" (sparse LU of M on the coarsest level), "jacobi"
    (coarse_sweeps damped-Jacobi sweeps with weight coarse_w from zero) or
    "auto" (jacobi where the coarsest level's smallest kh, omega times its
    spacing times the smallest slowness of the model, is at least 2.5 --
    there damped Jacobi contracts every mode -- else exact).
    rho: density of Eq. (1) (None: constant density), injected to the coarse
    levels like the slowness; kh then uses the slowness m / sqrt(rho).
    """

    def __init__(self, m, h, omega, beta1, beta2, levels, nu1=2, nu2=2, wj=None, coarse="exact",
                 coarse_sweeps=2, coarse_w=0.8, rho=None):
        m = np.asarray(m, dtype=np.float64)
        rl = None if rho is None else np.asarray(rho, dtype=np.float64)
        if levels < 1:
            raise ValueError("levels must be >= 1")
        if wj is None:
            wj = [0.8] * (levels - 1)
        wj = list(wj)
        if len(wj) < levels - 1:
            raise ValueError("need one Jacobi weight per smoothing level")
        self.nu1, self.nu2 = nu1, nu2
        self.wj = wj
        self.shapes, self.M, self.D, self.P, self.R = [], [], [], [], []
        ml, hl = m, h
        for l in range(levels):
            self.shapes.append(ml.shape)
            Ml = operator_M(ml, hl, omega, beta1, beta2, rl)
            self.M.append(Ml)
            self.D.append(Ml.diagonal())
            if l < levels - 1:
                cs = coarse_shape(ml.shape)
                self.P.append(prolongation(cs, ml.shape))
                self.R.append(restriction(cs, ml.shape))
                ml, hl = inject(ml), 2 * hl
                rl = None if rl is None else inject(rl)
        if coarse == "auto":
            me = m if rho is None else m / np.sqrt(np.asarray(rho, dtype=np.float64))
            kh_min = omega * h * 2.0 ** (levels - 1) * float(np.min(me))
            coarse = "jacobi" if levels > 1 and kh_min >= 2.5 else "exact"
        self.coarse = coarse
        self.coarse_sweeps, self.coarse_w = coarse_sweeps, coarse_w
        self.coarse_lu = factor_superlu(self.M[-1]) if coarse == "exact" else None
        self.levels = levels

    def smooth(self, l, u, b, sweeps):
        for _ in range(sweeps):
            u = u + self.wj[l] * (b - self.M[l] @ u) / self.D[l]
        return u

    def cycle(self, l, b):
        if l == self.levels - 1:
            if self.coarse == "exact":
                return self.coarse_lu.solve(b)
            u = np.zeros_like(b)
            for _ in range(self.coarse_sweeps):
                u = u + self.coarse_w * (b - self.M[l] @ u) / self.D[l]
            return u
        u = np.zeros_like(b)
        u = self.smooth(l, u, b, self.nu1)
        rc = self.R[l] @ (b - self.M[l] @ u)
        u = u + self.P[l] @ self.cycle(l + 1, rc)
        return self.smooth(l, u, b, self.nu2)

    def __call__(self, b):
        return self.cycle(0, np.asarray(b, dtype=np.complex128))


def vcycle_matrix(vc):
    """Dense matrix of the V-cycle built from its error-propagation form.

    For the two levels l, l+1 the error after one cycle is
    E_l = S_l^nu2 (I - P_l C_{l+1} R_l M_l) S_l^nu1 with S_l = I - w_l D_l^-1 M_l,
    where C_{l+1} is the coarse map (exact inverse on the coarsest level,
    else the coarser V-cycle's matrix). The V-cycle's matrix is then
    C_l = (I - E_l) M_l^-1. Dense; for tiny grids only.
    """
    Mc = vc.M[-1].toarray()
    if vc.coarse == "exact":
        C = np.linalg.inv(Mc)
    else:
        # k sweeps from zero: u = (I - S^k) M^-1 b with S = I - w D^-1 M
        S = np.eye(Mc.shape[0]) - vc.coarse_w * (Mc / vc.D[-1][:, None])
        C = (np.eye(Mc.shape[0]) - np.linalg.matrix_power(S, vc.coarse_sweeps)) @ np.linalg.inv(Mc)
    for l in range(vc.levels - 2, -1, -1):
        M = vc.M[l].toarray()
        n = M.shape[0]
        S = np.eye(n) - vc.wj[l] * (M / vc.D[l][:, None])
        cg = np.eye(n) - vc.P[l].toarray() @ C @ vc.R[l].toarray() @ M
        E = np.linalg.matrix_power(S, vc.nu2) @ cg @ np.linalg.matrix_power(S, vc.nu1)
        C = (np.eye(n) - E) @ np.linalg.inv(M)
    return C
