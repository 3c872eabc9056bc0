"""GPU parity on 3D grids (Eq. (1) with d = 3, constant density) against the
oracle, element by element on seeded inputs: the operators B and M on every
level, one damped-Jacobi sweep, the weighted restriction, the trilinear
prolongation, the V-cycle, point sources; then whole solves against the
oracle's direct (LU) solution and its own preconditioned BiCGSTAB iteration
counts, batch invariance, graph replay, the level plan, the calls a 3D model
refuses, and the benchmark's own 129^3 workload checked through the oracle's
operator. Shapes mix odd and even node counts and span several 64-wide tiles
with ragged tails.

Tolerances as for 2D: one stencil evaluation 1e-13 relative, a V-cycle
1e-11, a solve to relative residual 1e-8 within 1e-6 of the LU solution and
iteration counts within max(2, 5 %) of the oracle's."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
from oracle import krylov
from oracle import direct
import workloads

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-13
TOL_CYCLE = 1e-11

SHAPES3 = [((17, 21, 33), 25.0), ((16, 18, 20), 30.0), ((9, 12, 65), 20.0)]


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
    c.set_model(torch.from_numpy(np.ascontiguousarray(m)), h)
    return c


def iters_close(a, b):
    return abs(a - b) <= max(2, int(0.05 * max(a, b)))


@pytest.mark.parametrize("shape,h", SHAPES3)
def test_3d_operator_on_every_level(hz, shape, h):
    import torch
    m = random_model(shape, 1)
    c = ctx_for(hz, m, h)
    f, alpha, beta = 7.0, 0.03, (1.0, 0.5)
    om = 2 * np.pi * f
    L = c.plan(f)[0]
    ml = m
    for l in range(L):
        shp = ml.shape
        assert shp == c.level_shape(l)
        x = workloads.random_vectors(2, int(np.prod(shp)), seed=10 + l)
        xt = torch.from_numpy(x.reshape((2,) + shp)).cuda()
        hl = h * 2 ** l
        yB = to_np(c.apply("B", l, f, xt, alpha=alpha, beta=beta)).reshape(2, -1)
        yM = to_np(c.apply("M", l, f, xt, alpha=alpha, beta=beta)).reshape(2, -1)
        B = op.operator_B(ml, hl, om, alpha)
        M = op.operator_M(ml, hl, om, *beta)
        for k in range(2):
            assert rel(yB[k], B @ x[k]) < TOL_STEP
            assert rel(yM[k], M @ x[k]) < TOL_STEP
        ml = mg.inject(ml)


@pytest.mark.parametrize("shape,h", SHAPES3)
def test_3d_smoother_restriction_prolongation(hz, shape, h):
    import torch
    m = random_model(shape, 2)
    c = ctx_for(hz, m, h)
    f, beta, w = 5.0, (1.0, 0.5), 0.7
    om = 2 * np.pi * f
    n = int(np.prod(shape))
    cs = mg.coarse_shape(shape)
    b = workloads.random_vectors(2, n, seed=3)
    u = workloads.random_vectors(2, n, seed=4)
    e = workloads.random_vectors(2, int(np.prod(cs)), seed=8)
    M = op.operator_M(m, h, om, *beta)
    D = M.diagonal()
    R = mg.restriction(cs, shape)
    P = mg.prolongation(cs, shape)
    bt = torch.from_numpy(b.reshape((2,) + shape)).cuda()
    ut = torch.from_numpy(u.reshape((2,) + shape)).cuda()
    out = to_np(c.smooth(0, f, bt, ut, w=w, beta=beta)).reshape(2, -1)
    out0 = to_np(c.smooth(0, f, bt, None, w=w, beta=beta)).reshape(2, -1)
    bc = to_np(c.restrict(0, f, bt, ut, beta=beta)).reshape(2, -1)
    up = to_np(c.prolong(0, torch.from_numpy(e.reshape((2,) + cs)).cuda(), ut)).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], u[k] + w * (b[k] - M @ u[k]) / D) < TOL_STEP
        assert rel(out0[k], w * b[k] / D) < TOL_STEP
        assert rel(bc[k], R @ (b[k] - M @ u[k])) < TOL_STEP
        assert rel(up[k], u[k] + P @ e[k]) < TOL_STEP


@pytest.mark.parametrize("shape,h,levels,nu", [((17, 17, 17), 40.0, 3, (2, 2)),
                                               ((16, 18, 20), 30.0, 2, (1, 1)),
                                               ((9, 12, 65), 20.0, 3, (2, 1)),
                                               ((20, 22, 70), 20.0, 3, (2, 2)),
                                               ((17, 13, 66), 20.0, 3, (1, 3))])
def test_3d_vcycle(hz, shape, h, levels, nu):
    """One V-cycle against the oracle's: the marching sweeps on grids whose y
    rows do not fill the last block of four, whose z-planes end in a short
    chunk, with even node counts (the coarse grid ends a fine spacing short)
    and more than one 62-column strip, the first post-sweep forming u + P e
    (or both post-sweeps in one march, then a third sweep of its own)."""
    import torch
    m = random_model(shape, 9)
    c = ctx_for(hz, m, h)
    f, beta = 6.0, (1.0, 0.5)
    wj = [0.8, 0.6][:levels - 1]
    vc = mg.VCycle(m, h, 2 * np.pi * f, beta[0], beta[1], levels, nu[0], nu[1], wj)
    n = int(np.prod(shape))
    b = workloads.random_vectors(2, n, seed=11)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((2,) + shape)).cuda(), levels=levels, nu=nu, beta=beta,
                          jacobi_w_level=wj, coarse="exact")).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


def test_3d_point_sources(hz):
    w = workloads.model_3d_layered(9, 10, 11, h=15.0, nshots=3)
    c = ctx_for(hz, w.m, w.h)
    b = to_np(c.point_rhs_3d([s[0] for s in w.src], [s[1] for s in w.src], [s[2] for s in w.src],
                             amp=[1.0, 2.0 - 1.0j, 0.5j]))
    for k, (iz, iy, ix) in enumerate(w.src):
        ref = op.point_source(w.shape, w.h, [(iz * w.shape[1] + iy) * w.shape[2] + ix], [[1.0, 2.0 - 1.0j, 0.5j][k]])
        assert np.array_equal(b[k].ravel(), ref)


def test_3d_solve_matches_direct_and_oracle_iterations(hz):
    """Layered 33 x 25 x 41 box (h = 20 m), 3 shots x 2 frequencies in one
    batch, planned levels and weights: every wavefield against its LU
    solution, the relative residual, and the first shot's iteration count
    against the oracle's BiCGSTAB with the same V-cycle."""
    import torch
    w = workloads.model_3d_layered(33, 25, 41, h=20.0, nshots=3, freqs=(3.0, 5.0))
    c = ctx_for(hz, w.m, w.h)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b1 = c.point_rhs_3d(iz, iy, ix)
    b = torch.stack([b1] * len(w.freqs)).contiguous()
    u, info = c.solve(w.freqs, w.alpha, b, tol=1e-8)
    u = to_np(u)
    ns = len(w.src)
    for fi, f in enumerate(w.freqs):
        om = 2 * np.pi * f
        B = op.operator_B(w.m, w.h, om, w.alpha)
        lu = direct.factor_superlu(B)
        L, wj = c.plan(f)
        vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
        for s in range(ns):
            st, it, rr = info[fi * ns + s]
            assert st == hz.HZ_RHS_CONVERGED and rr <= 1e-8
            bn = op.point_source(w.shape, w.h, [(iz[s] * w.shape[1] + iy[s]) * w.shape[2] + ix[s]])
            assert rel(u[fi, s].ravel(), lu.solve(bn)) < 1e-6
            if s == 0:
                _, it_o, _, st_o = krylov.bicgstab(B, bn, vc, tol=1e-8, maxit=2000)
                assert st_o == krylov.CONVERGED and iters_close(it, it_o), (f, it, it_o)


def test_3d_batch_invariance_bitwise(hz):
    """A right-hand side gives the same bits alone and inside a batch."""
    import torch
    w = workloads.model_3d_layered(17, 19, 21, h=25.0, nshots=4, freqs=(3.0, 4.0))
    c = ctx_for(hz, w.m, w.h)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b = c.point_rhs_3d(iz, iy, ix)
    u_all, info_all = c.solve(w.freqs, w.alpha, torch.stack([b, b.flip(0)]).contiguous(), tol=1e-10)
    u_one, info_one = c.solve([4.0], w.alpha, b[1:2][None].contiguous(), tol=1e-10)
    assert torch.equal(u_all[1, 2], u_one[0, 0])  # b.flip(0)[2] == b[1]
    assert info_all[4 + 2][1] == info_one[0][1]


def test_3d_refusals(hz):
    """What a 3D model does not take: the 2D source and receiver calls, the
    exact 1D preconditioner, an axis below three nodes; a 2D model refuses
    the 3D sources."""
    import torch
    w = workloads.model_3d_layered(9, 9, 9, h=30.0, nshots=1, freqs=(3.0,))
    c = ctx_for(hz, w.m, w.h)
    b = c.point_rhs_3d([0], [4], [4])[None].contiguous()
    with pytest.raises(hz.HzError) as e:
        c.solve(w.freqs, w.alpha, b, precond="exact")
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.point_rhs([0], [4])
    assert e.value.code == hz.HZ_ERR_ARG
    d_obs = torch.zeros((1, 1, 1), dtype=torch.complex128)
    with pytest.raises(hz.HzError) as e:
        c.misfit(w.freqs, w.alpha, [(0, 4)], [(0, 5)], d_obs, 0.0)
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.set_model(torch.from_numpy(np.full((2, 9, 9), 1 / 2000.0)), 30.0)
    assert e.value.code == hz.HZ_ERR_ARG
    c2 = ctx_for(hz, np.full((9, 9), 1 / 2000.0), 30.0)
    with pytest.raises(hz.HzError) as e:
        c2.point_rhs_3d([0], [1], [1])
    assert e.value.code == hz.HZ_ERR_ARG


def test_3d_vcycle_with_smoothed_coarsest_level(hz):
    """The coarsest level smoothed by damped-Jacobi sweeps instead of solved
    (the form taken where its smallest kh is large), against the oracle."""
    import torch
    shape, h, levels, f = (17, 17, 17), 60.0, 3, 12.0
    m = random_model(shape, 21)
    c = ctx_for(hz, m, h)
    wj = [0.6, 0.4]
    vc = mg.VCycle(m, h, 2 * np.pi * f, 1.0, 0.5, levels, 2, 2, wj, coarse="jacobi", coarse_sweeps=3)
    b = workloads.random_vectors(2, int(np.prod(shape)), seed=23)
    out = to_np(c.precond(f, torch.from_numpy(b.reshape((2,) + shape)).cuda(), levels=levels, nu=(2, 2),
                          jacobi_w_level=wj, coarse="jacobi", coarse_sweeps=3)).reshape(2, -1)
    for k in range(2):
        assert rel(out[k], vc(b[k])) < TOL_CYCLE


def test_3d_unpreconditioned_solve(hz):
    """No preconditioner on a small, damped 3D box: converges to the LU solution."""
    w = workloads.model_3d_layered(9, 11, 13, h=40.0, nshots=1, freqs=(2.0,))
    c = ctx_for(hz, w.m, w.h)
    (iz, iy, ix), = w.src
    b = c.point_rhs_3d([iz], [iy], [ix])
    u, info = c.solve([2.0], 0.2, b[None].contiguous(), precond="none", tol=1e-10, maxit=5000)
    assert info[0][0] == hz.HZ_RHS_CONVERGED
    B = op.operator_B(w.m, w.h, 2 * np.pi * 2.0, 0.2)
    bn = op.point_source(w.shape, w.h, [(iz * w.shape[1] + iy) * w.shape[2] + ix])
    assert rel(to_np(u)[0, 0].ravel(), direct.solve_superlu(B, bn)) < 1e-8


@pytest.mark.parametrize("f", [2.0, 6.0, 12.0])
def test_3d_plan_matches_oracle_plan(hz, f):
    """The library's level count and damped-Jacobi weights on a 3D grid are
    the oracle's plan (local Fourier analysis with dim = 3)."""
    from oracle import lfa
    w = workloads.model_3d_layered(65, 33, 49, h=20.0, nshots=1)
    c = ctx_for(hz, w.m, w.h)
    L, wj = c.plan(f)
    Lo, wo = lfa.plan(w.shape, w.h, 2 * np.pi * f, float(w.m.min()), float(w.m.max()), 1.0, 0.5)
    assert L == Lo and np.allclose(wj, wo, rtol=0, atol=1e-15), (L, wj, Lo, wo)


def test_3d_graph_replay_bitwise(hz):
    """Iterations replayed from captured HIP graphs on a 3D model give the
    same bits and iteration counts as iterations issued one by one."""
    import torch
    w = workloads.model_3d_layered(17, 21, 19, h=25.0, nshots=3, freqs=(3.0, 5.0))
    c = ctx_for(hz, w.m, w.h)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b1 = c.point_rhs_3d(iz, iy, ix)
    b = torch.stack([b1] * len(w.freqs)).contiguous()
    ref, info_ref = c.solve(w.freqs, w.alpha, b, tol=1e-10, graphs=False)
    for _ in range(2):
        u, info = c.solve(w.freqs, w.alpha, b, tol=1e-10, graphs=True)
        assert torch.equal(u, ref)
        assert [i[:2] for i in info] == [i[:2] for i in info_ref]


def test_3d_benchmark_workload_residuals(hz):
    """The 3D benchmark's own workload (129^3, h = 20 m, 8 shots x 3/5 Hz, in
    the launch configuration the benchmark times): every right-hand side
    converges, the iteration counts of two shots per frequency are the
    oracle's (stored by tests/golden/make_3d_oracle_iterations.py) within
    max(2, 5 %), and the oracle's operator confirms ||b - B u|| / ||b|| <= 2 tol
    for each of them (a property that holds at any size)."""
    import torch
    w = workloads.model_3d_layered(129, 129, 129, h=20.0, nshots=8, freqs=(3.0, 5.0))
    c = ctx_for(hz, w.m, w.h)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b1 = c.point_rhs_3d(iz, iy, ix)
    b = torch.stack([b1] * len(w.freqs)).contiguous()
    print(f"[3d-bench-workload] solving {b.shape[0] * b.shape[1]} right-hand sides on {w.shape}", flush=True)
    u, info = c.solve(w.freqs, w.alpha, b, tol=1e-8)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    # iteration counts of the shots the oracle ran to convergence (tests/golden)
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "l3d_oracle_iterations.json")) as fh:
        gold = json.load(fh)
    for fi, f in enumerate(w.freqs):
        for s, it_o in zip(gold["shots"], gold["freqs"][str(f)]["iterations"]):
            it = info[fi * len(w.src) + s][1]
            assert iters_close(it, it_o), (f, s, it, it_o)
    u, bh = to_np(u), to_np(b)
    for fi, f in enumerate(w.freqs):
        B = op.operator_B(w.m, w.h, 2 * np.pi * f, w.alpha)
        for s in range(len(w.src)):
            r = bh[fi, s].ravel() - B @ u[fi, s].ravel()
            assert np.linalg.norm(r) <= 2e-8 * np.linalg.norm(bh[fi, s]), (f, s)


@pytest.mark.parametrize("m", [30, 5])
def test_3d_gmres_matches_direct_and_oracle(hz, m):
    """GMRES(m) with the V-cycle on a 3D box: the wavefields against LU and
    the iteration count against the oracle's GMRES(m) with the same V-cycle."""
    import torch
    w = workloads.model_3d_layered(17, 21, 25, h=25.0, nshots=2, freqs=(4.0,))
    c = ctx_for(hz, w.m, w.h)
    iz, iy, ix = ([s[a] for s in w.src] for a in range(3))
    b = c.point_rhs_3d(iz, iy, ix)[None].contiguous()
    u, info = c.solve(w.freqs, w.alpha, b, krylov="gmres", gmres_m=m, tol=1e-8)
    u = to_np(u)
    om = 2 * np.pi * w.freqs[0]
    B = op.operator_B(w.m, w.h, om, w.alpha)
    L, wj = c.plan(w.freqs[0])
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
    for s in range(len(w.src)):
        st, it, rr = info[s]
        assert st == hz.HZ_RHS_CONVERGED and rr <= 1e-8
        bn = op.point_source(w.shape, w.h, [(iz[s] * w.shape[1] + iy[s]) * w.shape[2] + ix[s]])
        assert rel(u[0, s].ravel(), direct.solve_superlu(B, bn)) < 1e-6
        if s == 0:
            _, it_o, _, st_o = krylov.gmres(B, bn, vc, m=m, tol=1e-8, maxit=2000)
            assert st_o == krylov.CONVERGED and iters_close(it, it_o), (it, it_o)
