"""ORACLE (test infrastructure only): gradient of the misfit J(m) by the
adjoint-state method, Born (linearised) modelling, and the Gauss-Newton
normal operator.

Eq. (4) defines J(m) = sum |u_obs - u_cal(m)|^2 + lam sum m^2 over shots,
receivers and frequencies; Eq. (7) gives its gradient through the Frechet
derivative G = du_cal/dm, and Eq. (8)-(9) the Gauss-Newton Hessian
Re[G^H G] + lam I and update. The paper prints Eq. (7) without the factor 2,
with a transpose where the complex data need a conjugate transpose, and with
the residual sign folded into Delta u; the oracle computes the exact
derivative of J as written (readings listed in the design doc):

* u = B^-1 b per (shot, frequency); only the diagonal of B depends on m:
  dB_ii/dm_i = delta_i = j omega g_i / h - 2 omega^2 (1 - j alpha) w_i m_i
  (the absorbing boundary term included; with a fixed density rho of Eq. (1)
  that term carries sqrt(rho_i));
* du/dm_i = -B^-1 e_i delta_i u_i, so the Born data of a perturbation dm are
  G dm = -P B^-1 (delta * u * dm);
* with the data residual res = P u - d_obs and the adjoint field
  mu = B^-T P^T conj(res) (= B^-1 P^T conj(res), B being symmetric),
  dJ/dm_i = -2 Re[ sum delta_i u_i mu_i ] + 2 lam m_i;
* the Gauss-Newton operator of J is H v = 2 Re[G^H G v] + 2 lam v.

All solves are direct (SuperLU), as the paper does for its observed data.
"""

import numpy as np

from .operator import operator_B, stencil_parts, point_source
from .direct import factor_superlu


def diag_derivative(m, h, omega, alpha, rho=None):
    """delta_i = d(B_ii)/d(m_i) for every node (flattened)."""
    m = np.asarray(m, dtype=np.float64)
    _, g, w = stencil_parts(m.shape)
    mf = m.ravel()
    if rho is not None:
        g = g * np.sqrt(np.asarray(rho, dtype=np.float64).ravel())
    return 1j * omega * g / h - 2.0 * omega ** 2 * (1.0 - 1j * alpha) * w * mf


class Survey:
    """Shots (point sources), receivers (nodes) and frequencies on a grid."""

    def __init__(self, shape, h, freqs, alpha, src_nodes, rec_nodes, src_amps=None, rho=None):
        self.rho = None if rho is None else np.asarray(rho, dtype=np.float64)  # density of Eq. (1), fixed
        self.shape = tuple(shape)
        self.h = float(h)
        self.freqs = [float(f) for f in freqs]
        self.alpha = float(alpha)
        self.src = [int(s) for s in src_nodes]
        self.rec = np.asarray(rec_nodes, dtype=np.int64)
        self.amps = src_amps

    def rhs(self):
        """Weighted right-hand sides, [nsrc, n]."""
        amps = self.amps if self.amps is not None else [1.0] * len(self.src)
        return np.array([point_source(self.shape, self.h, [s], [a]) for s, a in zip(self.src, amps)])


def forward(m, sv):
    """Wavefields u[f][s] (n,) and the LU factors per frequency."""
    b = sv.rhs()
    us, lus = [], []
    for f in sv.freqs:
        lu = factor_superlu(operator_B(m, sv.h, 2 * np.pi * f, sv.alpha, sv.rho))
        lus.append(lu)
        us.append(np.array([lu.solve(bs) for bs in b]))
    return us, lus


def data(m, sv):
    """Modelled receiver data [nfreq, nsrc, nrec]."""
    us, _ = forward(m, sv)
    return np.array([u[:, sv.rec] for u in us])


def misfit(m, sv, d_obs, lam):
    d = data(m, sv)
    r = d - d_obs
    return float(np.sum(r.real ** 2 + r.imag ** 2) + lam * np.sum(np.asarray(m) ** 2))


def gradient(m, sv, d_obs, lam):
    """(J, dJ/dm with the shape of m) by the adjoint-state method."""
    m = np.asarray(m, dtype=np.float64)
    n = m.size
    us, lus = forward(m, sv)
    J = lam * float(np.sum(m ** 2))
    g = np.zeros(n)
    for fi, f in enumerate(sv.freqs):
        delta = diag_derivative(m, sv.h, 2 * np.pi * f, sv.alpha, sv.rho)
        for s in range(len(sv.src)):
            u = us[fi][s]
            res = u[sv.rec] - d_obs[fi, s]
            J += float(np.sum(res.real ** 2 + res.imag ** 2))
            src = np.zeros(n, dtype=np.complex128)
            np.add.at(src, sv.rec, np.conj(res))
            mu = lus[fi].solve(src)
            g += -2.0 * np.real(delta * u * mu)
    g += 2.0 * lam * m.ravel()
    return J, g.reshape(m.shape)


def born(m, sv, dm):
    """G dm: linearised data [nfreq, nsrc, nrec] of a slowness perturbation."""
    m = np.asarray(m, dtype=np.float64)
    us, lus = forward(m, sv)
    out = []
    for fi, f in enumerate(sv.freqs):
        delta = diag_derivative(m, sv.h, 2 * np.pi * f, sv.alpha, sv.rho)
        rows = []
        for s in range(len(sv.src)):
            w = lus[fi].solve(-delta * us[fi][s] * np.asarray(dm).ravel())
            rows.append(w[sv.rec])
        out.append(rows)
    return np.array(out)


def born_adjoint(m, sv, dd):
    """G^H dd as a complex model-space vector (G acting on complex
    perturbations), so that <G v, w> = <v, G^H w> holds exactly; the real
    part is what a real slowness update uses."""
    m = np.asarray(m, dtype=np.float64)
    us, lus = forward(m, sv)
    n = m.size
    acc = np.zeros(n, dtype=np.complex128)
    for fi, f in enumerate(sv.freqs):
        delta = diag_derivative(m, sv.h, 2 * np.pi * f, sv.alpha, sv.rho)
        for s in range(len(sv.src)):
            src = np.zeros(n, dtype=np.complex128)
            np.add.at(src, sv.rec, dd[fi, s])
            # B^-H src = conj(B^-1 conj(src)) since B is symmetric
            z = np.conj(lus[fi].solve(np.conj(src)))
            acc += -np.conj(delta * us[fi][s]) * z
    return acc.reshape(m.shape)


def gauss_newton_apply(m, sv, v, lam):
    """H v = 2 Re[G^H G v] + 2 lam v."""
    gv = born(m, sv, v)
    return 2.0 * np.real(born_adjoint(m, sv, gv)) + 2.0 * lam * np.asarray(v)


def gauss_newton_step(m, sv, d_obs, lam, cg_iters, cg_tol=0.0):
    """One Gauss-Newton update (Eq. (9)): solve H dm = -g by conjugate
    gradients (the paper solves its Gauss-Newton system with CG because the
    Hessian is dense) from dm = 0, at most cg_iters iterations or until
    ||residual|| <= cg_tol ||g||; return (m + dm, dm, J(m), iterations)."""
    m = np.asarray(m, dtype=np.float64)
    J, g = gradient(m, sv, d_obs, lam)
    x = np.zeros_like(m)
    r = -g.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    g2 = rr
    it = 0
    while it < cg_iters and rr > (cg_tol ** 2) * g2:
        Hp = gauss_newton_apply(m, sv, p, lam)
        a = rr / float(np.sum(p * Hp))
        x = x + a * p
        r = r - a * Hp
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return m + x, x, J, it
