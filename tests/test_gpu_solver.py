"""GPU parity of the whole solve against the oracle: wavefields against the
oracle's direct (LU) solution, iteration counts against the oracle's own
preconditioned Krylov solve, the true residual recomputed by the oracle from
the GPU's u, batch invariance, failure paths, the misfit of Eq. (4), and the
full 401 x 801 x 256-right-hand-side configuration checked on sampled shots.

Tolerances: the solver stops at relative residual tol; the wavefield error
against LU must stay below 1e-6 (relative, 2-norm) at tol = 1e-8, and
iteration counts may differ from the oracle's by max(2, 5 %) because the two
sides round differently (fused multiply-adds, reduction order); on the full
configuration, whose solves run up to 270 iterations, by max(3, 8 %) per shot
and 4 % over the three sampled shots together."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
from oracle import krylov
from oracle import direct
from oracle import lfa
from oracle import misfit as omisfit
import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_np(t):
    return t.detach().cpu().numpy()


def iters_close(a, b):
    return abs(a - b) <= max(2, int(0.05 * max(a, b)))


def make_ctx(hz, m, h):
    import torch
    c = hz.Context(0)
    c.set_model(torch.from_numpy(np.asarray(m)), h)
    return c


def test_c1_1d_three_layers_exact_preconditioner(hz):
    import torch
    w = workloads.model_1d_layers()
    c = make_ctx(hz, w.m, w.h)
    f = w.freqs[0]
    om = 2 * np.pi * f
    b = c.point_rhs([0], w.src)
    u, info = c.solve([f], w.alpha, b[None], precond="exact", tol=w.tol)
    st, it, rr = info[0]
    assert st == hz.HZ_RHS_CONVERGED and rr <= w.tol
    B = op.operator_B(w.m, w.h, om, w.alpha)
    bn = op.point_source(w.shape, w.h, w.src)
    assert np.array_equal(to_np(b)[0], bn)
    ulu = direct.solve_superlu(B, bn)
    ug = to_np(u)[0, 0]
    assert rel(ug, ulu) < 1e-6
    assert np.linalg.norm(bn - B @ ug) / np.linalg.norm(bn) <= 2 * w.tol
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 1)
    _, it_o, _, st_o = krylov.bicgstab(B, bn, vc, tol=w.tol, maxit=1000)
    assert st_o == krylov.CONVERGED and iters_close(it, it_o), (it, it_o)


@pytest.mark.parametrize("sign", [-1.0, 1.0])
@pytest.mark.parametrize("tol", [1e-8, 1e-12])
def test_c2_lens_vcycle(hz, sign, tol):
    w = workloads.model_2d_lens(sign=sign)
    c = make_ctx(hz, w.m, w.h)
    f = w.freqs[0]
    om = 2 * np.pi * f
    b = c.point_rhs([0], [w.src[0] % w.shape[1]])
    u, info = c.solve([f], w.alpha, b[None], levels=4, nu=(2, 2), jacobi_w_level=[0.8] * 3, tol=tol)
    st, it, rr = info[0]
    assert st == hz.HZ_RHS_CONVERGED and rr <= tol
    B = op.operator_B(w.m, w.h, om, w.alpha)
    bn = op.point_source(w.shape, w.h, w.src)
    ulu = direct.solve_superlu(B, bn)
    ug = to_np(u)[0, 0].ravel()
    err = rel(ug, ulu)
    assert err < (1e-6 if tol == 1e-8 else 1e-9), err
    assert np.linalg.norm(bn - B @ ug) / np.linalg.norm(bn) <= 2 * tol
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 4, 2, 2, [0.8] * 3, coarse="auto")
    _, it_o, _, _ = krylov.bicgstab(B, bn, vc, tol=tol, maxit=500)
    assert iters_close(it, it_o), (it, it_o)


@pytest.mark.parametrize("krylov_name", ["bicgstab", "gmres"])
def test_plain_per_launch_path(hz, krylov_name):
    """The plain per-launch path (single kernels for every step, dense
    shadow residual, host readback every iteration) runs the same
    iteration as the fused batched path: the same wavefield to rounding
    (both against LU), the oracle's iteration count, and GMRES too."""
    w = workloads.model_2d_lens(sign=-1.0)
    c = make_ctx(hz, w.m, w.h)
    f = w.freqs[0]
    om = 2 * np.pi * f
    b = c.point_rhs([0, 0], [100, 37])
    kw = dict(levels=4, nu=(2, 2), jacobi_w_level=[0.8] * 3, tol=1e-10, krylov=krylov_name)
    u0, i0 = c.solve([f], w.alpha, b[None], **kw)
    u1, i1 = c.solve([f], w.alpha, b[None], plain=True, **kw)
    B = op.operator_B(w.m, w.h, om, w.alpha)
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 4, 2, 2, [0.8] * 3, coarse="auto")
    for s, ix in enumerate((100, 37)):
        assert i0[s][0] == hz.HZ_RHS_CONVERGED and i1[s][0] == hz.HZ_RHS_CONVERGED
        bn = op.point_source(w.shape, w.h, [ix])
        ulu = direct.solve_superlu(B, bn)
        assert rel(to_np(u1)[0, s].ravel(), ulu) < 1e-8
        assert rel(to_np(u1)[0, s].ravel(), to_np(u0)[0, s].ravel()) < 1e-8
        assert iters_close(i1[s][1], i0[s][1])
        if krylov_name == "bicgstab":
            _, it_o, _, _ = krylov.bicgstab(B, bn, vc, tol=1e-10, maxit=500)
        else:
            _, it_o, _, _ = krylov.gmres(B, bn, vc, m=30, tol=1e-10, maxit=500)
        assert iters_close(i1[s][1], it_o), (i1[s][1], it_o)


def test_multi_frequency_multi_shot_batch(hz):
    """Several frequencies and shots in one batch, planned weights, each
    right-hand side against its own LU solution."""
    import torch
    w = workloads.model_2d_layered(nz=101, nx=201, h=20.0, nshots=5, freqs=(2.0, 4.0, 6.5))
    c = make_ctx(hz, w.m, w.h)
    ns = len(w.src)
    b1 = c.point_rhs([0] * ns, w.src)
    b = torch.stack([b1] * len(w.freqs))
    u, info = c.solve(w.freqs, w.alpha, b, tol=1e-8)
    u = to_np(u)
    for fi, f in enumerate(w.freqs):
        om = 2 * np.pi * f
        B = op.operator_B(w.m, w.h, om, w.alpha)
        lu = direct.factor_superlu(B)
        L, wj = lfa.plan(w.shape, w.h, om, w.m.min(), w.m.max(), 1.0, 0.5)
        vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
        for s in range(ns):
            st, it, rr = info[fi * ns + s]
            assert st == hz.HZ_RHS_CONVERGED and rr <= 1e-8
            bn = op.point_source(w.shape, w.h, [w.src[s]])
            assert rel(u[fi, s].ravel(), lu.solve(bn)) < 1e-6
            if s == 0:
                _, it_o, _, _ = krylov.bicgstab(B, bn, vc, tol=1e-8, maxit=2000)
                assert iters_close(it, it_o), (f, it, it_o)


def test_batch_invariance_bitwise(hz):
    """A right-hand side gives the same bits alone and inside a batch."""
    import torch
    w = workloads.model_2d_lens(n=129, h=15.0)
    c = make_ctx(hz, w.m, w.h)
    rng = np.random.default_rng(3)
    xs = rng.integers(0, 129, size=6)
    b = c.point_rhs([0] * 6, xs)
    u_all, info_all = c.solve([4.0, 6.0], 0.01, torch.stack([b, b.flip(0)]))
    u_one, info_one = c.solve([6.0], 0.01, b[2:3][None])
    assert torch.equal(u_all[1, 3], u_one[0, 0])  # b.flip(0)[3] == b[2]
    assert info_all[6 + 3][1] == info_one[0][1]
    u_one4, _ = c.solve([4.0], 0.01, b[4:5][None])
    assert torch.equal(u_all[0, 4], u_one4[0, 0])


@pytest.mark.parametrize("shape", [(129, 129), (65, 257)])
def test_launch_shape_invariance_bitwise(hz, shape):
    """The fused V-cycle kernels give the same bits for every launch shape
    (rows per wavefront), so the tuner's choice never changes a result."""
    import torch
    nz, nx = shape
    w = workloads.model_2d_layered(nz=nz, nx=nx, h=15.0, nshots=5, freqs=(4.0,))
    c = make_ctx(hz, w.m, w.h)
    b = c.point_rhs([0] * 5, w.src)[None]
    ref, info_ref = c.solve([4.0], 0.01, b, tol=1e-9, autotune=False)
    for ch in (2, 8, 64, 512):
        u, info = c.solve([4.0], 0.01, b, tol=1e-9, chunk_rows=ch)
        assert torch.equal(u, ref), ch
        assert [i[1] for i in info] == [i[1] for i in info_ref]
    u, _ = c.solve([4.0], 0.01, b, tol=1e-9, autotune=True)
    assert torch.equal(u, ref)


@pytest.mark.parametrize("nrhs,freqs", [(1, (5.0,)), (7, (3.0, 6.0, 9.0))])
def test_graph_replay_bitwise(hz, nrhs, freqs):
    """Iterations replayed from captured HIP graphs give the same bits and
    iteration counts as iterations issued one by one (several batch-size
    buckets as right-hand sides converge, and a second solve that captures
    its graphs again)."""
    import torch
    w = workloads.model_2d_layered(nz=97, nx=193, h=20.0, nshots=nrhs, freqs=freqs)
    c = make_ctx(hz, w.m, w.h)
    b1 = c.point_rhs([0] * nrhs, w.src)
    b = torch.stack([b1] * len(freqs)).contiguous()
    ref, info_ref = c.solve(freqs, 0.01, b, tol=1e-10, graphs=False)
    for _ in range(2):
        u, info = c.solve(freqs, 0.01, b, tol=1e-10, graphs=True)
        assert torch.equal(u, ref)
        assert [i[:2] for i in info] == [i[:2] for i in info_ref]


def test_unpreconditioned_path(hz):
    """No preconditioner: a small, heavily damped problem still converges."""
    w = workloads.model_2d_lens(n=33, h=60.0)
    c = make_ctx(hz, w.m, w.h)
    b = c.point_rhs([0], [16])
    u, info = c.solve([2.0], 0.2, b[None], precond="none", tol=1e-10, maxit=5000)
    assert info[0][0] == hz.HZ_RHS_CONVERGED
    B = op.operator_B(w.m, w.h, 2 * np.pi * 2.0, 0.2)
    assert rel(to_np(u)[0, 0].ravel(), direct.solve_superlu(B, op.point_source(w.shape, w.h, [16]))) < 1e-8


@pytest.mark.parametrize("shape", [(3, 3), (5, 5), (4, 7), (3,), (6,)])
def test_tiny_grids(hz, shape):
    """The smallest grids: one level (the dense exact inverse of M), and an
    even-count grid that can be halved once."""
    import torch
    rng = np.random.default_rng(4)
    m = 1.0 / rng.uniform(1500, 3000, size=shape)
    h, f = 50.0, 6.0
    c = make_ctx(hz, m, h)
    n = int(np.prod(shape))
    b = workloads.random_vectors(2, n, seed=2)
    ref = direct.solve_dense(op.operator_B(m, h, 2 * np.pi * f, 0.01), b.T).T
    for levels in sorted({1, lfa.max_levels(shape)}):
        u, info = c.solve([f], 0.01, torch.from_numpy(b.reshape((1, 2) + shape)), tol=1e-12, levels=levels)
        assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
        assert rel(to_np(u).reshape(2, -1), ref) <= 1e-9


def test_coarse_smoothing_solve_matches_direct(hz):
    """A batch mixing frequencies whose coarsest level is solved exactly and
    smoothed (coarse="auto") still converges to the direct solution."""
    import torch
    w = workloads.model_2d_layered(nz=65, nx=129, h=40.0, nshots=3, freqs=(1.0, 12.0))
    c = make_ctx(hz, w.m, w.h)
    b1 = c.point_rhs([0] * 3, w.src)
    b = torch.stack([b1, b1]).contiguous()
    u, info = c.solve(w.freqs, 0.01, b, tol=1e-10, coarse="auto", coarse_sweeps=8)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    bn = to_np(b1).reshape(3, -1)
    for k, f in enumerate(w.freqs):
        lu = direct.factor_superlu(op.operator_B(w.m, w.h, 2 * np.pi * f, 0.01))
        ref = np.array([lu.solve(x) for x in bn])
        assert rel(to_np(u[k]).reshape(3, -1), ref) <= 1e-7


def test_sparse_and_dense_shadow_residuals(hz):
    """r^ = b is kept as a list when b has at most 256 nonzeros (inner
    products with r^ formed from the list) and streamed as a vector
    otherwise. Point sources, 256 and 257 nonzeros, a dense b and b = 0 in one
    batch: every slot converges to the direct solution, the point source in
    the oracle's iteration count, and a slot gives the same bits alone."""
    import torch
    w = workloads.model_2d_lens(n=65, h=30.0)
    c = make_ctx(hz, w.m, w.h)
    rng = np.random.default_rng(11)
    n = w.shape[0] * w.shape[1]
    bs = np.zeros((5, n), dtype=np.complex128)
    bs[0] = op.point_source(w.shape, w.h, [20])
    for k, nnz in ((1, 256), (2, 257)):
        pos = rng.choice(n, size=nnz, replace=False)
        bs[k, pos] = rng.standard_normal(nnz) + 1j * rng.standard_normal(nnz)
    bs[3] = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = torch.from_numpy(bs.reshape((1, 5) + w.shape)).cuda()
    f = 5.0
    u, info = c.solve([f], 0.01, b, tol=1e-10)
    om = 2 * np.pi * f
    B = op.operator_B(w.m, w.h, om, 0.01)
    lu = direct.factor_superlu(B)
    for k in range(4):
        assert info[k][0] == hz.HZ_RHS_CONVERGED, (k, info[k])
        assert rel(to_np(u[0, k]).ravel(), lu.solve(bs[k])) <= 1e-7, k
    assert info[4] == (hz.HZ_RHS_CONVERGED, 0, 0.0)
    L, wj = lfa.plan(w.shape, w.h, om, w.m.min(), w.m.max(), 1.0, 0.5)
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
    _, it_o, _, _ = krylov.bicgstab(B, bs[0], vc, tol=1e-10, maxit=2000)
    assert iters_close(info[0][1], it_o), (info[0][1], it_o)
    for k in (0, 1, 2):
        u1, info1 = c.solve([f], 0.01, b[:, k:k + 1].contiguous(), tol=1e-10)
        assert torch.equal(u1[0, 0], u[0, k]), k
        assert info1[0][1] == info[k][1]


@pytest.mark.parametrize("restart_at,graphs", [(5, False), (6, False), (6, True)])
def test_forced_restart_converges(hz, restart_at, graphs):
    """BiCGSTAB's breakdown restart (r^ = r, p = v = 0), forced after
    iteration 5 (which leaves its term of the iterate pending: it is added
    before the restart) and 6: r^ becomes a dense vector; point sources
    (sparse r^ before the restart) and a dense b still converge to the
    direct solution."""
    import torch
    w = workloads.model_2d_lens(n=65, h=30.0)
    c = make_ctx(hz, w.m, w.h)
    rng = np.random.default_rng(5)
    n = w.shape[0] * w.shape[1]
    bs = np.zeros((3, n), dtype=np.complex128)
    bs[0] = op.point_source(w.shape, w.h, [20])
    bs[1] = op.point_source(w.shape, w.h, [33 * 65 + 40])
    bs[2] = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = torch.from_numpy(bs.reshape((1, 3) + w.shape)).cuda()
    f = 5.0
    u, info = c.solve([f], 0.01, b, tol=1e-10, restart_at=restart_at, graphs=graphs)
    lu = direct.factor_superlu(op.operator_B(w.m, w.h, 2 * np.pi * f, 0.01))
    u_ref, info_ref = c.solve([f], 0.01, b, tol=1e-10)
    for k in range(3):
        assert info[k][0] == hz.HZ_RHS_CONVERGED, (k, info[k])
        assert info[k][1] > restart_at
        assert info[k][2] <= 1e-10
        assert rel(to_np(u[0, k]).ravel(), lu.solve(bs[k])) <= 1e-7, k
        # the restart costs iterations but the result is the same solution
        assert rel(to_np(u[0, k]), to_np(u_ref[0, k])) <= 1e-7
    # the restarted recurrences differ from the unforced ones
    assert any(info[k][1] != info_ref[k][1] for k in range(3))


def test_kernel_timing_classes(hz):
    """hz_timing_start/read: every launch of a timed class is counted (one
    pre-smoothing launch of each kind, one operator apply on s^ and one update
    per BiCGSTAB iteration, two post-smoothing launches per iteration, the
    coarser levels' launches), the times are positive, untimed classes stay at
    zero, timing does not change the result, and a class past the last one is
    refused. With point sources r^ is a sparse list and no operator pass on p^
    is made (the pre-smoothing kernels form B p^); a dense right-hand side
    takes one per iteration for <r^, B p^>."""
    import torch
    w = workloads.model_2d_layered(nz=97, nx=193, h=20.0, nshots=3, freqs=(4.0,))
    c = make_ctx(hz, w.m, w.h)
    b = c.point_rhs([0] * 3, w.src)[None]
    ref, info_ref = c.solve([4.0], 0.01, b, tol=1e-9)
    c.timing_start(["apply", "apply_s", "update", "prolong", "presmooth_s", "levels"])
    u, info = c.solve([4.0], 0.01, b, tol=1e-9)
    t = {k: c.timing_read(k) for k in hz.HZ_KERNEL}
    c.timing_start([])
    assert torch.equal(u, ref)
    slot_iters = sum(i[1] for i in info)
    for k in ("presmooth_s", "apply_s", "update"):
        assert t[k][0] >= max(i[1] for i in info) and t[k][1] > 0.0, (k, t[k])
    assert t["apply"] == (0, 0.0)
    assert t["prolong"][0] == 2 * t["presmooth_s"][0]
    assert t["levels"][0] > t["prolong"][0] and t["levels"][1] > 0.0
    assert t["presmooth"] == (0, 0.0) and t["coarse"] == (0, 0.0)
    assert slot_iters >= t["update"][0]
    g = torch.Generator().manual_seed(5)
    bd = torch.complex(torch.randn((1, 2) + w.shape, generator=g, dtype=torch.float64),
                       torch.randn((1, 2) + w.shape, generator=g, dtype=torch.float64)).cuda()
    c.timing_start(["apply", "presmooth_s"])
    _, info_d = c.solve([4.0], 0.01, bd, tol=1e-9)
    td = {k: c.timing_read(k) for k in ("apply", "presmooth_s")}
    c.timing_start([])
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info_d)
    assert td["apply"][0] == td["presmooth_s"][0] >= max(i[1] for i in info_d) and td["apply"][1] > 0.0, td
    with pytest.raises(hz.HzError) as e:
        c.timing_start([len(hz.HZ_KERNEL)])
    assert e.value.code == hz.HZ_ERR_ARG


def test_empty_batch(hz):
    import torch
    w = workloads.model_2d_lens(n=33, h=40.0)
    c = make_ctx(hz, w.m, w.h)
    b = torch.empty((1, 0) + w.shape, dtype=torch.complex128, device="cuda")
    u, info = c.solve([5.0], 0.01, b)
    assert u.shape == b.shape and info == []


def test_failure_paths(hz):
    import torch
    w = workloads.model_2d_lens(n=65, h=30.0)
    c = make_ctx(hz, w.m, w.h)
    b = c.point_rhs([0, 0, 0], [10, 20, 30])
    b[1].zero_()
    b[2, 5, 5] = complex(float("nan"), 0.0)
    u, info = c.solve([5.0], 0.01, b[None], tol=1e-10)
    assert info[0][0] == hz.HZ_RHS_CONVERGED
    assert info[1] == (hz.HZ_RHS_CONVERGED, 0, 0.0)
    assert not torch.any(u[0, 1] != 0)
    assert info[2][0] == hz.HZ_RHS_NONFINITE
    # iteration cap
    u, info = c.solve([5.0], 0.01, b[:1][None], tol=1e-14, maxit=1)
    assert info[0][0] == hz.HZ_RHS_MAXIT and info[0][1] == 1
    # argument errors
    with pytest.raises(hz.HzError) as e:
        c.solve([-1.0], 0.01, b[:1][None])
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.solve([5.0], 0.01, b[:1][None], levels=12)
    assert e.value.code == hz.HZ_ERR_SHAPE
    with pytest.raises(hz.HzError) as e:
        c.solve([5.0], 0.01, b[:1][None], beta=(1.0, 0.0))
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.point_rhs([0], [65])
    assert e.value.code == hz.HZ_ERR_ARG
    bad = torch.from_numpy(w.m.copy())
    bad[3, 3] = -1.0
    with pytest.raises(hz.HzError) as e:
        c.set_model(bad, w.h)
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.solve([5.0], 0.01, b[:1][None])
    assert e.value.code == hz.HZ_ERR_STATE


def test_misfit_matches_oracle(hz):
    import torch
    true = workloads.model_2d_layered(nz=65, nx=129, h=25.0, nshots=4, freqs=(2.0, 3.5))
    start = workloads.model_2d_layered(nz=65, nx=129, h=25.0, nshots=4, freqs=(2.0, 3.5), seed=1)
    src = [(0, s) for s in true.src]
    rec = [(0, r) for r in range(0, 129, 8)]
    rec_nodes = [r[1] for r in rec]
    lam = 1e-3
    d_obs = np.zeros((2, 4, len(rec)), dtype=complex)
    d_cal = np.zeros_like(d_obs)
    for fi, f in enumerate(true.freqs):
        om = 2 * np.pi * f
        lu_t = direct.factor_superlu(op.operator_B(true.m, true.h, om, true.alpha))
        lu_s = direct.factor_superlu(op.operator_B(start.m, start.h, om, start.alpha))
        for s, (iz, ix) in enumerate(src):
            bn = op.point_source(true.shape, true.h, [ix])
            d_obs[fi, s] = omisfit.sample(lu_t.solve(bn), rec_nodes)
            d_cal[fi, s] = omisfit.sample(lu_s.solve(bn), rec_nodes)
    J_o = omisfit.misfit(d_obs, d_cal, start.m, lam)
    c = make_ctx(hz, start.m, start.h)
    J, dc, info = c.misfit(true.freqs, true.alpha, src, rec, torch.from_numpy(d_obs), lam, tol=1e-10)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    assert rel(to_np(dc), d_cal) < 1e-7
    assert abs(J - J_o) <= 1e-7 * J_o


def test_full_size_batched_configuration(hz):
    """401 x 801 grid, 64 surface shots x {3, 5, 8, 12} Hz = 256 right-hand
    sides in one batch (the benchmark's launch configuration, default plan
    and coarse policy). Every one of the 256 returned wavefields has its
    true residual recomputed with the oracle's sparse B; shots 0, 31 and 63
    of every frequency are checked against LU and their iteration counts
    against the oracle's own BiCGSTAB with the same V-cycle
    (tests/golden/c3_oracle_iterations.json, written by the oracle alone)."""
    import json
    import os
    import torch
    w = workloads.model_2d_layered()
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_oracle_iterations.json")))
    assert gold["coarse_policy"] == "auto" and gold["tol"] == 1e-8
    c = make_ctx(hz, w.m, w.h)
    ns = len(w.src)
    b1 = c.point_rhs([0] * ns, w.src)
    b = torch.stack([b1] * len(w.freqs))
    u, info = c.solve(w.freqs, w.alpha, b, tol=1e-8)
    assert all(i[0] == hz.HZ_RHS_CONVERGED and i[2] <= 1e-8 for i in info), info
    U = to_np(u).reshape(len(w.freqs), ns, -1)
    bn = to_np(b1).reshape(ns, -1)
    for fi, f in enumerate(w.freqs):
        om = 2 * np.pi * f
        g = gold["freqs"][str(f)]
        L, wj = c.plan(f)
        assert L == g["levels"] and np.allclose(wj, g["jacobi_w"], rtol=0, atol=1e-15)
        B = op.operator_B(w.m, w.h, om, w.alpha)
        # true residual of all 64 wavefields from the oracle's operator
        R = (bn - (B @ U[fi].T).T)
        rr = np.linalg.norm(R, axis=1) / np.linalg.norm(bn, axis=1)
        gpu_rr = np.array([info[fi * ns + s][2] for s in range(ns)])
        assert rr.max() <= 1.01e-8, (f, rr.max())
        assert np.allclose(rr, gpu_rr, rtol=1e-3, atol=0), (f, rr, gpu_rr)
        lu = direct.factor_superlu(B)
        its = []
        for k, s in enumerate(gold["shots"]):
            ref = lu.solve(op.point_source(w.shape, w.h, [w.src[s]]))
            assert rel(U[fi, s], ref) < 1e-6, (f, s)
            it = info[fi * ns + s][1]
            its.append(it)
            # a single long BiCGSTAB run moves by several iterations with the
            # rounding order alone (two valid contraction orders of the same
            # kernels gave 99 and 93 here), so per shot the bound is wider
            # than in the short solves, and the three shots' sum is checked
            assert abs(it - g["iterations"][k]) <= max(3, int(0.08 * max(it, g["iterations"][k]))), \
                (f, s, it, g["iterations"][k])
        assert abs(sum(its) - sum(g["iterations"])) <= 0.04 * sum(g["iterations"]), (f, its, g["iterations"])


@pytest.mark.parametrize("m,tol", [(30, 1e-8), (5, 1e-10)])
def test_gmres_matches_oracle(hz, m, tol):
    """GMRES(m) (the paper's data-modelling engine) with the V-cycle: the
    wavefield against LU and the inner-step count against the oracle's
    GMRES(m) (modified Gram-Schmidt there, delayed classical Gram-Schmidt
    twice here: the same mathematics)."""
    w = workloads.model_2d_lens(sign=-1.0)
    c = make_ctx(hz, w.m, w.h)
    f = w.freqs[0]
    om = 2 * np.pi * f
    b = c.point_rhs([0, 0], [100, 37])
    u, info = c.solve([f], w.alpha, b[None], krylov="gmres", gmres_m=m, levels=4, nu=(2, 2),
                      jacobi_w_level=[0.8] * 3, tol=tol, maxit=3000)
    B = op.operator_B(w.m, w.h, om, w.alpha)
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 4, 2, 2, [0.8] * 3, coarse="auto")
    for s, ix in enumerate((100, 37)):
        st, it, rr = info[s]
        assert st == hz.HZ_RHS_CONVERGED and rr <= tol
        bn = op.point_source(w.shape, w.h, [ix])
        ulu = direct.solve_superlu(B, bn)
        assert rel(to_np(u)[0, s].ravel(), ulu) < 1e-6
        _, it_o, _, st_o = krylov.gmres(B, bn, vc, m=m, tol=tol, maxit=3000)
        assert st_o == krylov.CONVERGED and iters_close(it, it_o), (it, it_o)


@pytest.mark.parametrize("m", [1, 2, 3, 7])
def test_gmres_short_restarts(hz, m):
    """GMRES(m) with short cycles, where the Arnoldi steps' delayed second
    pass meets the cycle's end at every few columns (m = 1: every column is
    completed by a cycle's closing pass): three shots against LU and the
    oracle's GMRES(m) iteration counts, with the planned V-cycle."""
    w = workloads.model_2d_lens(n=65, h=20.0)
    f, alpha = 6.0, 0.01
    om = 2 * np.pi * f
    c = make_ctx(hz, w.m, w.h)
    xs = [8, 32, 56]
    b = c.point_rhs([0] * 3, xs)
    u, info = c.solve([f], alpha, b[None], krylov="gmres", gmres_m=m, tol=1e-8, maxit=2000)
    L, wj = c.plan(f)
    B = op.operator_B(w.m, w.h, om, alpha)
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
    lu = direct.factor_superlu(B)
    for s, ix in enumerate(xs):
        st, it, rr = info[s]
        assert st == hz.HZ_RHS_CONVERGED and rr <= 1e-8, info[s]
        bn = op.point_source(w.shape, w.h, [ix])
        assert rel(to_np(u)[0, s].ravel(), lu.solve(bn)) < 1e-6
        _, it_o, _, st_o = krylov.gmres(B, bn, vc, m=m, tol=1e-8, maxit=2000)
        assert st_o == krylov.CONVERGED and iters_close(it, it_o), (m, ix, it, it_o)


@pytest.mark.parametrize("maxit", [4, 5, 6, 10])
def test_gmres_maxit_at_and_off_cycle_ends(hz, maxit):
    """An iteration limit that falls inside a cycle, on its last column
    (maxit = 5, 10 with m = 5) or one past it stops the solve after exactly
    maxit columns, with the iterate of those columns: its true residual is
    the oracle's GMRES(5) residual after maxit columns."""
    w = workloads.model_2d_lens(n=65, h=20.0)
    f, alpha = 6.0, 0.01
    om = 2 * np.pi * f
    c = make_ctx(hz, w.m, w.h)
    b = c.point_rhs([0], [32])
    u, info = c.solve([f], alpha, b[None], krylov="gmres", gmres_m=5, tol=1e-14, maxit=maxit)
    st, it, rr = info[0]
    assert st == hz.HZ_RHS_MAXIT and it == maxit, info[0]
    L, wj = c.plan(f)
    B = op.operator_B(w.m, w.h, om, alpha)
    vc = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
    bn = op.point_source(w.shape, w.h, [32])
    x_o, it_o, rr_o, st_o = krylov.gmres(B, bn, vc, m=5, tol=1e-14, maxit=maxit)
    assert st_o == krylov.MAXIT and it_o == maxit
    # a few columns of a well-conditioned minimisation: the two residuals agree closely
    assert abs(rr - rr_o) <= 1e-6 * rr_o, (rr, rr_o)
    assert rel(to_np(u)[0, 0].ravel(), x_o) < 1e-8


def test_gmres_batch_invariance_bitwise(hz):
    """A GMRES right-hand side gives the same bits alone and inside a batch
    of slots that finish at different Arnoldi steps."""
    import torch
    w = workloads.model_2d_lens(n=129, h=15.0)
    c = make_ctx(hz, w.m, w.h)
    rng = np.random.default_rng(5)
    xs = rng.integers(0, 129, size=6)
    b = c.point_rhs([0] * 6, xs)
    kw = dict(krylov="gmres", gmres_m=7)
    u_all, info_all = c.solve([4.0, 6.0], 0.01, torch.stack([b, b.flip(0)]), **kw)
    u_one, info_one = c.solve([6.0], 0.01, b[2:3][None], **kw)
    assert torch.equal(u_all[1, 3], u_one[0, 0])  # b.flip(0)[3] == b[2]
    assert info_all[6 + 3][1] == info_one[0][1]
    u_one4, _ = c.solve([4.0], 0.01, b[4:5][None], **kw)
    assert torch.equal(u_all[0, 4], u_one4[0, 0])
    assert len({i[1] for i in info_all}) > 1  # the slots stop at different steps


def test_gmres_unpreconditioned_and_maxit(hz):
    w = workloads.model_2d_lens(n=33, h=60.0)
    c = make_ctx(hz, w.m, w.h)
    b = c.point_rhs([0], [16])
    u, info = c.solve([2.0], 0.2, b[None], krylov="gmres", gmres_m=40, precond="none", tol=1e-10,
                      maxit=4000)
    assert info[0][0] == hz.HZ_RHS_CONVERGED
    B = op.operator_B(w.m, w.h, 2 * np.pi * 2.0, 0.2)
    bn = op.point_source(w.shape, w.h, [16])
    assert rel(to_np(u)[0, 0].ravel(), direct.solve_superlu(B, bn)) < 1e-8
    _, it_o, _, _ = krylov.gmres(B, bn, None, m=40, tol=1e-10, maxit=4000)
    assert iters_close(info[0][1], it_o), (info[0][1], it_o)
    u, info = c.solve([2.0], 0.2, b[None], krylov="gmres", gmres_m=10, tol=1e-14, maxit=7)
    assert info[0][0] == hz.HZ_RHS_MAXIT and info[0][1] == 7


def test_paper_comparisons_small(hz):
    """The comparisons the paper makes, on a small lens: every combination of
    BiCGSTAB / GMRES(30) with the V-cycle preconditioner at shifts (1, 0.5)
    and (1, 1) converges to the direct solution; the preconditioner cuts the
    operator applications of BiCGSTAB against the unpreconditioned solve."""
    import torch
    w = workloads.model_2d_lens(n=65, h=20.0)
    f = 6.0
    c = make_ctx(hz, w.m, w.h)
    xs = [8, 32, 56]
    b = c.point_rhs([0] * 3, xs)
    A = op.operator_B(w.m, w.h, 2 * np.pi * f, 0.01)
    lu = direct.factor_superlu(A)
    bn = to_np(b).reshape(3, -1)
    ref = np.array([lu.solve(x) for x in bn])
    ops = {}
    for kr in ("bicgstab", "gmres"):
        for pre, beta in (("mg", (1.0, 0.5)), ("mg", (1.0, 1.0)), ("none", (1.0, 0.5))):
            u, info = c.solve([f], 0.01, b[None], krylov=kr, precond=pre, beta=beta, tol=1e-9, maxit=4000)
            ops[(kr, pre, beta)] = np.mean([i[1] for i in info]) * (2 if kr == "bicgstab" else 1)
            if kr == "gmres" and pre == "none":
                continue  # restarted GMRES without a preconditioner may stall; it is only reported
            assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info), (kr, pre, beta, info)
            assert rel(to_np(u).reshape(3, -1), ref) <= 1e-6, (kr, pre, beta)
    assert ops[("bicgstab", "mg", (1.0, 0.5))] < ops[("bicgstab", "none", (1.0, 0.5))]
    assert ops[("gmres", "mg", (1.0, 0.5))] < ops[("bicgstab", "none", (1.0, 0.5))]
