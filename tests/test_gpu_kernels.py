"""GPU parity of each step of the path against the oracle, element by element,
on seeded inputs: the operator B and the shifted Laplacian M on every level,
one damped-Jacobi sweep, the weighted restriction, the prolongation, the
coarse (dense-inverse) solve, the 1D exact tridiagonal solve and the whole
V-cycle. Grids span several 64-wide tiles with ragged tails."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
import workloads

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-13   # one stencil evaluation: rounding of ~10 flops per entry
TOL_CYCLE = 1e-11  # a V-cycle: a few dozen sweeps and a dense coarse solve


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()


def random_model(shape, seed, lo=1500.0, hi=4500.0):
    rng = np.random.default_rng(seed)
    return 1.0 / rng.uniform(lo, hi, size=shape)


def ctx_for(hz, m, h):
    import torch
    c = hz.Context(0)
    c.set_model(torch.from_numpy(m), h)
    return c


def level_models(m, levels):
    out = [m]
    for _ in range(levels - 1):
        out.append(mg.inject(out[-1]))
    return out


# odd node counts (grids share both ends) and even ones (the last fine node
# of an even axis is interpolated from the last coarse node)
SHAPES = [((33, 65), 25.0), ((65, 33), 25.0), ((17, 129), 20.0), ((257,), 10.0),
          ((34, 66), 25.0), ((21, 40), 30.0), ((256,), 10.0)]


@pytest.mark.parametrize("shape,h", SHAPES)
def test_operator_on_every_level(hz, shape, h):
    import torch
    m = random_model(shape, 1)
    c = ctx_for(hz, m, h)
    f, alpha, beta = 7.0, 0.03, (1.0, 0.5)
    om = 2 * np.pi * f
    L = c.plan(f)[0]
    ms = level_models(m, L)
    for l in range(L):
        shp = ms[l].shape
        x = workloads.random_vectors(3, int(np.prod(shp)), seed=10 + l)
        xt = torch.from_numpy(x.reshape((3,) + shp)).cuda()
        hl = h * 2 ** l
        yB = to_np(c.apply("B", l, f, xt, alpha=alpha, beta=beta)).reshape(3, -1)
        yM = to_np(c.apply("M", l, f, xt, alpha=alpha, beta=beta)).reshape(3, -1)
        B = op.operator_B(ms[l], hl, om, alpha)
        M = op.operator_M(ms[l], hl, om, *beta)
        for k in range(3):
            assert rel(yB[k], B @ x[k]) < TOL_STEP
            assert rel(yM[k], M @ x[k]) < TOL_STEP


@pytest.mark.parametrize("shape,h", SHAPES)
def test_smoother_sweep(hz, shape, h):
    import torch
    m = random_model(shape, 2)
    c = ctx_for(hz, m, h)
    f, beta, w = 5.0, (1.0, 0.5), 0.7
    om = 2 * np.pi * f
    n = int(np.prod(shape))
    b = workloads.random_vectors(2, n, seed=3)
    u = workloads.random_vectors(2, n, seed=4)
    M = op.operator_M(m, h, om, *beta)
    D = M.diagonal()
    bt = torch.from_numpy(b.reshape((2,) + shape)).cuda()
    ut = torch.from_numpy(u.reshape((2,) + shape)).cuda()
    out = to_np(c.smooth(0, f, bt, ut, w=w, beta=beta)).reshape(2, -1)
    out0 = to_np(c.smooth(0, f, bt, None, w=w, beta=beta)).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], u[k] + w * (b[k] - M @ u[k]) / D) < TOL_STEP
        assert rel(out0[k], w * b[k] / D) < TOL_STEP


@pytest.mark.parametrize("shape,h", SHAPES)
def test_restriction_and_prolongation(hz, shape, h):
    import torch
    m = random_model(shape, 5)
    c = ctx_for(hz, m, h)
    f, beta = 6.0, (1.0, 0.5)
    om = 2 * np.pi * f
    n = int(np.prod(shape))
    cs = mg.coarse_shape(shape)
    b = workloads.random_vectors(2, n, seed=6)
    u = workloads.random_vectors(2, n, seed=7)
    e = workloads.random_vectors(2, int(np.prod(cs)), seed=8)
    M = op.operator_M(m, h, om, *beta)
    R = mg.restriction(cs, shape)
    P = mg.prolongation(cs, shape)
    bc = to_np(c.restrict(0, f, torch.from_numpy(b.reshape((2,) + shape)).cuda(),
                          torch.from_numpy(u.reshape((2,) + shape)).cuda(), beta=beta)).reshape(2, -1)
    up = to_np(c.prolong(0, torch.from_numpy(e.reshape((2,) + cs)).cuda(),
                         torch.from_numpy(u.reshape((2,) + shape)).cuda())).reshape(2, -1)
    for k in range(2):
        assert rel(bc[k], R @ (b[k] - M @ u[k])) < TOL_STEP
        assert rel(up[k], u[k] + P @ e[k]) < TOL_STEP


@pytest.mark.parametrize("shape,h,levels,nu", [
    ((33, 65), 25.0, 5, (2, 2)), ((33, 65), 25.0, 3, (1, 1)), ((65, 33), 25.0, 4, (2, 0)),
    ((17, 129), 20.0, 3, (3, 2)), ((257,), 10.0, 6, (2, 2)), ((101, 201), 10.0, 3, (2, 2)),
    ((34, 66), 25.0, 4, (2, 2)), ((60, 100), 20.0, 4, (2, 2)), ((34, 66), 25.0, 3, (1, 1)),
    ((256,), 10.0, 6, (2, 2))])
def test_vcycle(hz, shape, h, levels, nu):
    import torch
    m = random_model(shape, 9)
    c = ctx_for(hz, m, h)
    f, beta = 9.0, (1.0, 0.5)
    om = 2 * np.pi * f
    wj = [0.8, 0.6, 0.4, 0.3, 0.3][:levels - 1]
    vc = mg.VCycle(m, h, om, beta[0], beta[1], levels, nu[0], nu[1], wj)
    n = int(np.prod(shape))
    b = workloads.random_vectors(3, n, seed=11)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((3,) + shape)).cuda(), levels=levels,
                          nu=nu, beta=beta, jacobi_w_level=wj, coarse="exact")).reshape(3, -1)
    for k in range(3):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


@pytest.mark.parametrize("mode,f", [("jacobi", 3.0), ("auto", 12.0), ("auto", 1.0)])
def test_vcycle_coarse_smoothing(hz, mode, f):
    """The coarsest level smoothed by damped-Jacobi sweeps instead of solved;
    "auto" smooths it only where its smallest kh is >= 2.5 (12 Hz here,
    not 1 Hz)."""
    import torch
    shape, h = (65, 129), 40.0
    m = random_model(shape, 13)
    c = ctx_for(hz, m, h)
    L = c.plan(f)[0]
    wj = [0.8, 0.7, 0.5, 0.3, 0.3][:L - 1]
    hc = h * 2 ** (L - 1)
    kh_min = 2 * np.pi * f * hc * m.min()
    jac = mode == "jacobi" or kh_min >= 2.5
    assert jac == (mode == "jacobi" or f == 12.0)
    vc = mg.VCycle(m, h, 2 * np.pi * f, 1.0, 0.5, L, 2, 2, wj, coarse="jacobi" if jac else "exact", coarse_sweeps=5)
    b = workloads.random_vectors(2, m.size, seed=14)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((2,) + shape)).cuda(), jacobi_w_level=wj,
                          coarse=mode, coarse_sweeps=5)).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


def test_vcycle_uses_the_lfa_plan(hz):
    """Without fixed weights the library plans them; the oracle's plan gives
    the same V-cycle."""
    import torch
    from oracle import lfa
    w = workloads.model_2d_layered(nz=101, nx=201, h=40.0)
    c = ctx_for(hz, w.m, w.h)
    f = 4.0
    L, wj = lfa.plan(w.shape, w.h, 2 * np.pi * f, w.m.min(), w.m.max(), 1.0, 0.5)
    assert c.plan(f) == (L, wj)
    vc = mg.VCycle(w.m, w.h, 2 * np.pi * f, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
    b = workloads.random_vectors(2, w.m.size, seed=12)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((2,) + w.shape)).cuda())).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


@pytest.mark.parametrize("shape,h", [((21, 37), 30.0), ((9, 9), 50.0), ((129,), 10.0)])
def test_single_level_dense_inverse(hz, shape, h):
    """levels = 1: the preconditioner is the exact inverse of M (the coarse
    solve kernel on the whole grid)."""
    import torch
    m = random_model(shape, 13)
    c = ctx_for(hz, m, h)
    f, beta = 11.0, (1.0, 0.5)
    vc = mg.VCycle(m, h, 2 * np.pi * f, beta[0], beta[1], 1)
    n = int(np.prod(shape))
    b = workloads.random_vectors(9, n, seed=14)  # more than one block group of right-hand sides
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((9,) + shape)).cuda(), levels=1)).reshape(9, -1)
    for k in range(9):
        assert rel(out[k], vc(b[k])) < 1e-11


@pytest.mark.parametrize("n,h,f", [(1001, 5.0, 10.0), (257, 10.0, 30.0), (2048 + 1, 2.5, 10.0)])
def test_exact_tridiagonal_1d(hz, n, h, f):
    import torch
    w = workloads.model_1d_layers(n=n, h=h)
    c = ctx_for(hz, w.m, h)
    try:
        out = c.precond(f, torch.from_numpy(workloads.random_vectors(4, n, seed=15)).cuda(), precond="exact")
    except hz.HzError as e:
        assert n > 2048 and e.code == hz.HZ_ERR_ARG
        return
    b = workloads.random_vectors(4, n, seed=15)
    M = op.operator_M(w.m, h, 2 * np.pi * f, 1.0, 0.5)
    out = to_np(out)
    for k in range(4):
        assert rel(M @ out[k], b[k]) < 1e-12
