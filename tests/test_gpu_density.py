"""GPU parity of the variable-density operator of Eq. (1) against the oracle:
B and M on every level (densities injected like the slowness), one
damped-Jacobi sweep, the weighted restriction, the whole V-cycle and its plan
for the slowness m / sqrt(rho), the solve in 1D and 2D with BiCGSTAB and
GMRES against the oracle's LU and its Krylov iteration counts, a batch of
shots and frequencies, the allocation-free solve, the adjoint-state gradient,
the constant-density identity B_rho=c(m) = c B(m / sqrt(c)) on the full
401 x 801 grid, the return to constant density, and on 3D boxes the
operators, a sweep, the restriction, the V-cycle, a solve and the gradient.

Tolerances as for constant density: one stencil evaluation 1e-13, a V-cycle
1e-11 (relative 2-norm); wavefields 1e-6 against LU at tol = 1e-8; iteration
counts within max(2, 5 %) of the oracle's."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
from oracle import krylov
from oracle import direct
from oracle import lfa
from oracle import gradient as og
import workloads

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-13
TOL_CYCLE = 1e-11


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy()


def iters_close(a, b):
    return abs(a - b) <= max(2, int(0.05 * max(a, b)))


def random_model(shape, seed):
    rng = np.random.default_rng(seed)
    return 1.0 / rng.uniform(1500.0, 4500.0, size=shape), rng.uniform(0.5, 2.5, size=shape)


def ctx(hz, m, h, rho=None):
    import torch
    c = hz.Context(0)
    c.set_model(torch.from_numpy(np.asarray(m)), h)
    if rho is not None:
        c.set_density(torch.from_numpy(np.asarray(rho)))
    return c


def injected(a, levels):
    out = [a]
    for _ in range(levels - 1):
        out.append(mg.inject(out[-1]))
    return out


SHAPES = [((33, 65), 25.0), ((65, 33), 25.0), ((34, 66), 25.0), ((21, 40), 30.0), ((257,), 10.0), ((256,), 10.0)]


@pytest.mark.parametrize("shape,h", SHAPES)
def test_density_operator_on_every_level(hz, shape, h):
    import torch
    m, rho = random_model(shape, 1)
    c = ctx(hz, m, h, rho)
    f, alpha, beta = 7.0, 0.03, (1.0, 0.5)
    om = 2 * np.pi * f
    L = c.plan(f)[0]
    ms, rs = injected(m, L), injected(rho, L)
    for l in range(L):
        shp = ms[l].shape
        x = workloads.random_vectors(3, int(np.prod(shp)), seed=10 + l)
        xt = torch.from_numpy(x.reshape((3,) + shp)).cuda()
        hl = h * 2 ** l
        yB = to_np(c.apply("B", l, f, xt, alpha=alpha, beta=beta)).reshape(3, -1)
        yM = to_np(c.apply("M", l, f, xt, alpha=alpha, beta=beta)).reshape(3, -1)
        B = op.operator_B(ms[l], hl, om, alpha, rs[l])
        M = op.operator_M(ms[l], hl, om, *beta, rho=rs[l])
        for k in range(3):
            assert rel(yB[k], B @ x[k]) < TOL_STEP
            assert rel(yM[k], M @ x[k]) < TOL_STEP


@pytest.mark.parametrize("shape,h", SHAPES)
def test_density_sweep_and_restriction(hz, shape, h):
    import torch
    m, rho = random_model(shape, 2)
    c = ctx(hz, m, h, rho)
    f, beta, w = 5.0, (1.0, 0.5), 0.7
    om = 2 * np.pi * f
    n = int(np.prod(shape))
    cs = mg.coarse_shape(shape)
    b = workloads.random_vectors(2, n, seed=3)
    u = workloads.random_vectors(2, n, seed=4)
    M = op.operator_M(m, h, om, *beta, rho=rho)
    D = M.diagonal()
    R = mg.restriction(cs, shape)
    bt = torch.from_numpy(b.reshape((2,) + shape)).cuda()
    ut = torch.from_numpy(u.reshape((2,) + shape)).cuda()
    sw = to_np(c.smooth(0, f, bt, ut, w=w, beta=beta)).reshape(2, -1)
    sw0 = to_np(c.smooth(0, f, bt, None, w=w, beta=beta)).reshape(2, -1)
    bc = to_np(c.restrict(0, f, bt, ut, beta=beta)).reshape(2, -1)
    for k in range(2):
        assert rel(sw[k], u[k] + w * (b[k] - M @ u[k]) / D) < TOL_STEP
        assert rel(sw0[k], w * b[k] / D) < TOL_STEP
        assert rel(bc[k], R @ (b[k] - M @ u[k])) < TOL_STEP


@pytest.mark.parametrize("shape,h,levels,nu,coarse", [
    ((33, 65), 25.0, 4, (2, 2), "exact"), ((101, 201), 10.0, 3, (2, 2), "exact"),
    ((34, 66), 25.0, 4, (2, 2), "jacobi"), ((60, 100), 20.0, 4, (1, 1), "exact"),
    ((257,), 10.0, 6, (2, 2), "exact"), ((256,), 10.0, 5, (2, 2), "jacobi")])
def test_density_vcycle(hz, shape, h, levels, nu, coarse):
    import torch
    m, rho = random_model(shape, 9)
    c = ctx(hz, m, h, rho)
    f, beta = 9.0, (1.0, 0.5)
    om = 2 * np.pi * f
    wj = [0.8, 0.6, 0.4, 0.3, 0.3][:levels - 1]
    vc = mg.VCycle(m, h, om, beta[0], beta[1], levels, nu[0], nu[1], wj, coarse=coarse, coarse_sweeps=3, rho=rho)
    b = workloads.random_vectors(3, m.size, seed=11)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((3,) + shape)).cuda(), levels=levels, nu=nu, beta=beta,
                          jacobi_w_level=wj, coarse=coarse, coarse_sweeps=3)).reshape(3, -1)
    for k in range(3):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


def test_density_plan_uses_the_density_slowness(hz):
    """The planned levels and weights are the oracle's plan for the range of
    m / sqrt(rho), and the planned cycle is the oracle's V-cycle."""
    import torch
    w = workloads.model_2d_layered(nz=101, nx=201, h=40.0)
    rho = workloads.gardner_density(w.m) ** 4  # a wide range: 1 to about 2
    me = op.effective_slowness(w.m, rho)
    c = ctx(hz, w.m, w.h, rho)
    f = 6.0
    L, wj = lfa.plan(w.shape, w.h, 2 * np.pi * f, me.min(), me.max(), 1.0, 0.5)
    assert c.plan(f) == (L, wj)
    assert lfa.plan(w.shape, w.h, 2 * np.pi * f, w.m.min(), w.m.max(), 1.0, 0.5) != (L, wj)
    vc = mg.VCycle(w.m, w.h, 2 * np.pi * f, 1.0, 0.5, L, 2, 2, wj, coarse="auto", rho=rho)
    b = workloads.random_vectors(2, w.m.size, seed=12)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((2,) + w.shape)).cuda())).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


@pytest.mark.parametrize("krylov_name", ["bicgstab", "gmres"])
def test_density_solve_lens(hz, krylov_name):
    w = workloads.model_2d_lens(sign=-1.0)
    rho = workloads.gardner_density(w.m)
    c = ctx(hz, w.m, w.h, rho)
    f = w.freqs[0]
    om = 2 * np.pi * f
    b = c.point_rhs([0, 0], [100, 37])
    kw = dict(levels=4, nu=(2, 2), jacobi_w_level=[0.8] * 3, tol=1e-8, krylov=krylov_name)
    u, info = c.solve([f], w.alpha, b[None], **kw)
    B = op.operator_B(w.m, w.h, om, w.alpha, rho)
    B0 = op.operator_B(w.m, w.h, om, w.alpha)
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 4, 2, 2, [0.8] * 3, coarse="auto", rho=rho)
    for s, ix in enumerate((100, 37)):
        st, it, rr = info[s]
        assert st == hz.HZ_RHS_CONVERGED and rr <= 1e-8
        bn = op.point_source(w.shape, w.h, [ix])
        ulu = direct.solve_superlu(B, bn)
        ug = to_np(u)[0, s].ravel()
        assert rel(ug, ulu) < 1e-6
        assert np.linalg.norm(bn - B @ ug) / np.linalg.norm(bn) <= 2e-8
        # the density changes the field: far from the constant-density one
        assert rel(ug, direct.solve_superlu(B0, bn)) > 1e-2
        if krylov_name == "bicgstab":
            _, it_o, _, _ = krylov.bicgstab(B, bn, vc, tol=1e-8, maxit=500)
        else:
            _, it_o, _, _ = krylov.gmres(B, bn, vc, m=30, tol=1e-8, maxit=500)
        assert iters_close(it, it_o), (it, it_o)


def test_density_fused_and_per_step_paths_agree(hz):
    """The fused 2D kernels with the density's coupling table and the
    per-step kernels (plain path) run the same iteration: wavefields to
    rounding and the same iteration counts (within the rounding allowance)."""
    import torch
    w = workloads.model_2d_layered(nz=201, nx=401, h=20.0, nshots=6, freqs=(4.0, 9.0))
    rho = workloads.gardner_density(w.m) ** 4
    c = ctx(hz, w.m, w.h, rho)
    b1 = c.point_rhs([0] * len(w.src), w.src)
    b = torch.stack([b1, b1])
    u0, i0 = c.solve(w.freqs, w.alpha, b, tol=1e-10)
    u1, i1 = c.solve(w.freqs, w.alpha, b, tol=1e-10, plain=True)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in i0 + i1)
    for k in range(len(i0)):
        assert iters_close(i0[k][1], i1[k][1]), (i0[k], i1[k])
    assert rel(to_np(u0), to_np(u1)) < 1e-8
    B = op.operator_B(w.m, w.h, 2 * np.pi * 9.0, w.alpha, rho)
    bn = op.point_source(w.shape, w.h, [w.src[3]])
    assert np.linalg.norm(bn - B @ to_np(u0)[1, 3].ravel()) / np.linalg.norm(bn) <= 2e-10


def test_density_multi_frequency_batch(hz):
    import torch
    w = workloads.model_2d_layered(nz=101, nx=201, h=20.0, nshots=5, freqs=(2.0, 4.0, 6.5))
    rho = workloads.gardner_density(w.m)
    c = ctx(hz, w.m, w.h, rho)
    ns = len(w.src)
    b1 = c.point_rhs([0] * ns, w.src)
    b = torch.stack([b1] * len(w.freqs))
    u, info = c.solve(w.freqs, w.alpha, b, tol=1e-8)
    u = to_np(u)
    for fi, f in enumerate(w.freqs):
        B = op.operator_B(w.m, w.h, 2 * np.pi * f, w.alpha, rho)
        lu = direct.factor_superlu(B)
        for s in (0, ns - 1):
            assert info[fi * ns + s][0] == hz.HZ_RHS_CONVERGED
            bn = op.point_source(w.shape, w.h, [w.src[s]])
            assert rel(u[fi, s].ravel(), lu.solve(bn)) < 1e-6


@pytest.mark.parametrize("precond", ["exact", "mg"])
def test_density_1d(hz, precond):
    w = workloads.model_1d_layers()
    rho = workloads.gardner_density(w.m)
    c = ctx(hz, w.m, w.h, rho)
    f = w.freqs[0]
    b = c.point_rhs([0], w.src)
    u, info = c.solve([f], w.alpha, b[None], precond=precond, tol=1e-10)
    assert info[0][0] == hz.HZ_RHS_CONVERGED
    B = op.operator_B(w.m, w.h, 2 * np.pi * f, w.alpha, rho)
    ulu = direct.solve_superlu(B, op.point_source(w.shape, w.h, w.src))
    assert rel(to_np(u)[0, 0], ulu) < 1e-8


def test_density_noalloc_matches_solve(hz):
    import torch
    w = workloads.model_2d_layered(nz=65, nx=129, h=20.0, nshots=4, freqs=(3.0, 5.0))
    c = ctx(hz, w.m, w.h, workloads.gardner_density(w.m))
    b1 = c.point_rhs([0] * len(w.src), w.src)
    b = torch.stack([b1, b1])
    u0, i0 = c.solve(w.freqs, w.alpha, b, tol=1e-10)
    u1, i1 = c.solve(w.freqs, w.alpha, b, noalloc=True, tol=1e-10)
    assert torch.equal(u0, u1) and i0 == i1


def test_density_gradient_matches_oracle(hz):
    import torch
    nz, nx, h = 33, 65, 30.0
    true = workloads.model_2d_layered(nz=nz, nx=nx, h=h, nshots=4, freqs=(2.0, 3.0, 4.5))
    start = workloads.model_2d_layered(nz=nz, nx=nx, h=h, nshots=4, freqs=(2.0, 3.0, 4.5), seed=3)
    rho = workloads.gardner_density(true.m)
    src = [(0, s) for s in true.src]
    rec = [(0, r) for r in range(0, nx, 3)] + [(nz - 1, nx // 2)]
    sv = og.Survey(true.shape, h, true.freqs, 0.02, true.src, [iz * nx + ix for iz, ix in rec], rho=rho)
    d_obs = og.data(true.m, sv)
    lam = 1e-3
    J_o, g_o = og.gradient(start.m, sv, d_obs, lam)
    c = ctx(hz, start.m, h, rho)
    J, g, info = c.gradient(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), lam, tol=1e-11)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    assert abs(J - J_o) <= 1e-8 * J_o
    g = g.cpu().numpy()
    assert np.linalg.norm(g - g_o) <= 1e-6 * np.linalg.norm(g_o)
    # the constant-density gradient is a different one
    J1, g1 = og.gradient(start.m, og.Survey(true.shape, h, true.freqs, 0.02, true.src, sv.rec), d_obs, lam)
    assert np.linalg.norm(g1 - g_o) > 1e-2 * np.linalg.norm(g_o)


def test_density_constant_identity_full_grid(hz):
    """rho = c everywhere on the 401 x 801 grid: B_rho(m) u = b is
    B(m / sqrt(c)) u = b / c, so the density solve and the constant-density
    solve of the scaled problem give the same wavefields (both to tol)."""
    import torch
    w = workloads.model_2d_layered(nshots=16, freqs=(5.0,))
    cst = 1.7
    c = ctx(hz, w.m, w.h, np.full(w.shape, cst))
    b = c.point_rhs([0] * len(w.src), w.src)
    u1, i1 = c.solve([5.0], w.alpha, b[None], tol=1e-10)
    c.set_model(torch.from_numpy(w.m / np.sqrt(cst)), w.h)
    u0, i0 = c.solve([5.0], w.alpha, (b / cst)[None], tol=1e-10)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in i0 + i1)
    assert rel(to_np(u1), to_np(u0)) < 1e-8
    # the true residual of sampled shots, recomputed by the oracle
    B = op.operator_B(w.m, w.h, 2 * np.pi * 5.0, w.alpha, np.full(w.shape, cst))
    for s in (0, 7, 15):
        bn = op.point_source(w.shape, w.h, [w.src[s]])
        assert np.linalg.norm(bn - B @ to_np(u1)[0, s].ravel()) / np.linalg.norm(bn) <= 2e-10


def test_density_cleared_and_refused(hz):
    import torch
    w = workloads.model_2d_lens(n=65, h=30.0)
    c = ctx(hz, w.m, w.h)
    b = c.point_rhs([0], [20])
    u0, _ = c.solve([5.0], w.alpha, b[None], tol=1e-10)
    rho = workloads.gardner_density(w.m) ** 4
    c.set_density(torch.from_numpy(rho))
    u1, _ = c.solve([5.0], w.alpha, b[None], tol=1e-10)
    assert rel(to_np(u1), to_np(u0)) > 1e-3
    c.set_density(None)
    u2, _ = c.solve([5.0], w.alpha, b[None], tol=1e-10)
    assert torch.equal(u2, u0)
    # a new model starts at constant density
    c.set_density(torch.from_numpy(rho))
    c.set_model(torch.from_numpy(w.m), w.h)
    u3, _ = c.solve([5.0], w.alpha, b[None], tol=1e-10)
    assert torch.equal(u3, u0)
    # invalid densities are refused and leave constant density
    for bad in (-1.0, 0.0, np.nan, np.inf):
        r = rho.copy()
        r[10, 7] = bad
        with pytest.raises(hz.HzError) as ei:
            c.set_density(torch.from_numpy(r))
        assert ei.value.code == hz.HZ_ERR_ARG
    u4, _ = c.solve([5.0], w.alpha, b[None], tol=1e-10)
    assert torch.equal(u4, u0)
    with pytest.raises(ValueError):
        c.set_density(torch.from_numpy(rho[:, :-1].copy()))
    c3 = hz.Context(0)
    c3.set_model(torch.full((9, 9, 9), 1 / 2000.0, dtype=torch.float64), 20.0)
    bad = np.ones((9, 9, 9))
    bad[4, 4, 4] = -2.0
    with pytest.raises(hz.HzError) as ei:
        c3.set_density(torch.from_numpy(bad))
    assert ei.value.code == hz.HZ_ERR_ARG


# ---------------------------------------------------------------- 3D grids (Eq. (1) with d = 3)

SHAPES3 = [((9, 11, 17), 40.0), ((10, 12, 16), 40.0)]


@pytest.mark.parametrize("shape,h", SHAPES3)
def test_3d_density_operator_and_sweep(hz, shape, h):
    import torch
    m, rho = random_model(shape, 21)
    c = ctx(hz, m, h, rho)
    f, alpha, beta, w = 5.0, 0.03, (1.0, 0.5), 0.7
    om = 2 * np.pi * f
    L = c.plan(f)[0]
    ms, rs = injected(m, L), injected(rho, L)
    for l in range(L):
        shp = ms[l].shape
        x = workloads.random_vectors(2, int(np.prod(shp)), seed=30 + l)
        xt = torch.from_numpy(x.reshape((2,) + shp)).cuda()
        hl = h * 2 ** l
        yB = to_np(c.apply("B", l, f, xt, alpha=alpha, beta=beta)).reshape(2, -1)
        yM = to_np(c.apply("M", l, f, xt, alpha=alpha, beta=beta)).reshape(2, -1)
        B = op.operator_B(ms[l], hl, om, alpha, rs[l])
        M = op.operator_M(ms[l], hl, om, *beta, rho=rs[l])
        for k in range(2):
            assert rel(yB[k], B @ x[k]) < TOL_STEP
            assert rel(yM[k], M @ x[k]) < TOL_STEP
    n = m.size
    b = workloads.random_vectors(2, n, seed=3)
    u = workloads.random_vectors(2, n, seed=4)
    M = op.operator_M(m, h, om, *beta, rho=rho)
    D = M.diagonal()
    bt = torch.from_numpy(b.reshape((2,) + shape)).cuda()
    ut = torch.from_numpy(u.reshape((2,) + shape)).cuda()
    sw = to_np(c.smooth(0, f, bt, ut, w=w, beta=beta)).reshape(2, -1)
    cs = mg.coarse_shape(shape)
    bc = to_np(c.restrict(0, f, bt, ut, beta=beta)).reshape(2, -1)
    R = mg.restriction(cs, shape)
    for k in range(2):
        assert rel(sw[k], u[k] + w * (b[k] - M @ u[k]) / D) < TOL_STEP
        assert rel(bc[k], R @ (b[k] - M @ u[k])) < TOL_STEP


@pytest.mark.parametrize("levels,nu", [(2, (2, 2)), (3, (2, 2)), (3, (1, 1))])
def test_3d_density_vcycle(hz, levels, nu):
    import torch
    shape, h = (17, 21, 33), 25.0
    m, rho = random_model(shape, 22)
    c = ctx(hz, m, h, rho)
    f, beta = 6.0, (1.0, 0.5)
    wj = [0.8, 0.6][:levels - 1]
    vc = mg.VCycle(m, h, 2 * np.pi * f, beta[0], beta[1], levels, nu[0], nu[1], wj, rho=rho)
    b = workloads.random_vectors(2, m.size, seed=11)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((2,) + shape)).cuda(), levels=levels, nu=nu, beta=beta,
                          jacobi_w_level=wj, coarse="exact")).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


def test_3d_density_solve_and_gradient(hz):
    """A layered 17 x 21 x 25 box with a Gardner density: 2 shots x 2
    frequencies against LU and the oracle's BiCGSTAB iteration count, then
    the adjoint-state gradient against the oracle's."""
    import torch
    w = workloads.model_3d_layered(17, 21, 25, h=25.0, nshots=2, freqs=(2.0, 3.5))
    rho = workloads.gardner_density(w.m)
    c = ctx(hz, w.m, w.h, rho)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b1 = c.point_rhs_3d(iz, iy, ix)
    b = torch.stack([b1] * len(w.freqs)).contiguous()
    u, info = c.solve(w.freqs, w.alpha, b, tol=1e-8)
    u = to_np(u)
    ns = len(w.src)
    nodes = [(iz[s] * w.shape[1] + iy[s]) * w.shape[2] + ix[s] for s in range(ns)]
    for fi, f in enumerate(w.freqs):
        om = 2 * np.pi * f
        B = op.operator_B(w.m, w.h, om, w.alpha, rho)
        lu = direct.factor_superlu(B)
        L, wj = c.plan(f)
        vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto", rho=rho)
        for s in range(ns):
            st, it, rr = info[fi * ns + s]
            assert st == hz.HZ_RHS_CONVERGED and rr <= 1e-8
            bn = op.point_source(w.shape, w.h, [nodes[s]])
            assert rel(u[fi, s].ravel(), lu.solve(bn)) < 1e-6
            if s == 0:
                _, it_o, _, _ = krylov.bicgstab(B, bn, vc, tol=1e-8, maxit=2000)
                assert iters_close(it, it_o), (f, it, it_o)
    start = workloads.model_3d_layered(17, 21, 25, h=25.0, nshots=2, freqs=(2.0, 3.5), seed=3)
    rec = [(0, y, x) for y in range(0, 21, 4) for x in range(0, 25, 4)]
    rec_nodes = [(a * w.shape[1] + b_) * w.shape[2] + c_ for a, b_, c_ in rec]
    sv = og.Survey(w.shape, w.h, w.freqs, w.alpha, nodes, rec_nodes, rho=rho)
    d_obs = og.data(w.m, sv)
    lam = 1e-3
    J_o, g_o = og.gradient(start.m, sv, d_obs, lam)
    c.set_model(torch.from_numpy(start.m), w.h)
    c.set_density(torch.from_numpy(rho))
    J, g, ginfo = c.gradient_3d(sv.freqs, sv.alpha, w.src, rec, torch.from_numpy(d_obs), lam, tol=1e-11)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in ginfo)
    assert abs(J - J_o) <= 1e-8 * J_o
    assert np.linalg.norm(g.cpu().numpy() - g_o) <= 1e-6 * np.linalg.norm(g_o)
