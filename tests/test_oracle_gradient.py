"""Pins of the oracle's adjoint-state gradient (Eq. (7)), Born modelling and
Gauss-Newton operator (Eq. (8)-(9)) against finite differences of J and of
the data, the Taylor remainder, the dot-product test and the symmetry and
positivity of the Gauss-Newton operator."""

import numpy as np

from oracle import gradient as og
import workloads


def _setup(n=(21, 33), h=40.0):
    nz, nx = n
    true = workloads.model_2d_layered(nz=nz, nx=nx, h=h, nshots=3, freqs=(2.0, 3.0))
    start = workloads.model_2d_layered(nz=nz, nx=nx, h=h, nshots=3, freqs=(2.0, 3.0), seed=5)
    rec = list(range(0, nx, 4)) + [nz * nx - 1]  # surface receivers and a corner
    sv = og.Survey(true.shape, h, true.freqs, 0.05, true.src, rec)
    d_obs = og.data(true.m, sv)
    return start.m, sv, d_obs


def _smooth_direction(shape, seed):
    v = workloads.smooth_random_vectors(1, shape, seed, sigma=2.0)[0].real
    return v.reshape(shape) / np.abs(v).max()


def test_gradient_matches_central_differences():
    m, sv, d_obs = _setup()
    lam = 1e-3 * 1e6  # regulariser comparable in size to the data misfit
    J, g = og.gradient(m, sv, d_obs, lam)
    assert np.isclose(J, og.misfit(m, sv, d_obs, lam), rtol=1e-12)
    for seed in (1, 2):
        v = _smooth_direction(m.shape, seed) * np.abs(m).max()
        eps = 1e-4
        fd = (og.misfit(m + eps * v, sv, d_obs, lam) - og.misfit(m - eps * v, sv, d_obs, lam)) / (2 * eps)
        an = float(np.sum(g * v))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_gradient_boundary_nodes():
    """Perturbing single boundary and corner nodes: the absorbing term's
    dependence on m is part of the gradient."""
    m, sv, d_obs = _setup()
    J, g = og.gradient(m, sv, d_obs, 0.0)
    nz, nx = m.shape
    for (iz, ix) in ((0, 5), (nz - 1, 7), (4, 0), (0, 0), (nz - 1, nx - 1)):
        v = np.zeros_like(m)
        v[iz, ix] = m[iz, ix]
        eps = 1e-5
        fd = (og.misfit(m + eps * v, sv, d_obs, 0.0) - og.misfit(m - eps * v, sv, d_obs, 0.0)) / (2 * eps)
        assert abs(fd - g[iz, ix] * v[iz, ix]) <= 1e-5 * abs(fd) + 1e-12 * J


def test_taylor_remainder_is_second_order():
    m, sv, d_obs = _setup()
    J, g = og.gradient(m, sv, d_obs, 0.0)
    v = _smooth_direction(m.shape, 3) * np.abs(m).max()
    rems = []
    for eps in (4e-3, 2e-3, 1e-3):
        rems.append(abs(og.misfit(m + eps * v, sv, d_obs, 0.0) - J - eps * float(np.sum(g * v))))
    assert 3.5 < rems[0] / rems[1] < 4.5 and 3.5 < rems[1] / rems[2] < 4.5, rems


def test_born_dot_product_and_finite_difference():
    m, sv, d_obs = _setup()
    rng = np.random.default_rng(0)
    v = rng.standard_normal(m.shape) + 1j * rng.standard_normal(m.shape)
    w = rng.standard_normal(d_obs.shape) + 1j * rng.standard_normal(d_obs.shape)
    lhs = np.vdot(w, og.born(m, sv, v))
    rhs = np.vdot(og.born_adjoint(m, sv, w), v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    dm = _smooth_direction(m.shape, 4) * np.abs(m).max()
    eps = 1e-5
    fd = (og.data(m + eps * dm, sv) - og.data(m - eps * dm, sv)) / (2 * eps)
    gb = og.born(m, sv, dm)
    assert np.linalg.norm(fd - gb) <= 1e-6 * np.linalg.norm(gb)


def test_gradient_equals_adjoint_of_born_on_residual():
    m, sv, d_obs = _setup()
    lam = 2.0
    _, g = og.gradient(m, sv, d_obs, lam)
    res = og.data(m, sv) - d_obs
    g2 = 2.0 * np.real(og.born_adjoint(m, sv, res)) + 2.0 * lam * m
    assert np.linalg.norm(g - g2) <= 1e-12 * np.linalg.norm(g)


def test_gauss_newton_operator_symmetric_positive():
    m, sv, d_obs = _setup((13, 17), 60.0)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(m.shape)
    w = rng.standard_normal(m.shape)
    lam = 1e-3
    Hv = og.gauss_newton_apply(m, sv, v, lam)
    Hw = og.gauss_newton_apply(m, sv, w, lam)
    assert abs(np.sum(Hv * w) - np.sum(v * Hw)) <= 1e-10 * abs(np.sum(Hv * w))
    assert np.sum(Hv * v) > 0


def test_gauss_newton_step_solves_the_normal_equations():
    """CG run to convergence solves H dm = -g (checked against the dense
    Gauss-Newton matrix assembled column by column); dm is a descent
    direction and lowers the quadratic model of J."""
    m, sv, d_obs = _setup((9, 13), 90.0)
    lam = 1e-2
    m1, dm, J0, it = og.gauss_newton_step(m, sv, d_obs, lam, cg_iters=400, cg_tol=1e-13)
    n = m.size
    H = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        H[:, k] = og.gauss_newton_apply(m, sv, e.reshape(m.shape), lam).ravel()
    _, g = og.gradient(m, sv, d_obs, lam)
    ref = np.linalg.solve(H, -g.ravel())
    assert np.linalg.norm(dm.ravel() - ref) <= 1e-7 * np.linalg.norm(ref)
    slope = float(np.sum(g * dm))
    assert slope < 0
    assert slope + 0.5 * float(dm.ravel() @ H @ dm.ravel()) < 0
    assert og.misfit(m + 1e-3 * dm, sv, d_obs, lam) < J0
