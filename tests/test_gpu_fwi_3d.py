"""GPU parity of the misfit (Eq. (4)), the adjoint-state gradient (Eq. (7))
and the Gauss-Newton step (Eq. (8)-(9)) on 3D models against the oracle
(direct solves), a finite-difference check on the GPU's own 3D misfit, and
the calls' refusals across dimensions.

Tolerances as for 2D: the solves stop at relative residual 1e-11 or 1e-12,
so wavefields carry errors of about 1e-10 relative; J must agree with the
oracle's to 1e-8 relative, the gradient and the update to 1e-6 (2-norm), the
gradient with central differences of the GPU misfit to 1e-5."""

import numpy as np
import pytest

from oracle import gradient as og
import workloads

pytestmark = pytest.mark.gpu


def _survey(shape=(13, 17, 21), h=40.0, nshots=4, freqs=(2.0, 3.5)):
    nz, ny, nx = shape
    true = workloads.model_3d_layered(nz, ny, nx, h=h, nshots=nshots, freqs=freqs, nlayers=4)
    start = workloads.model_3d_layered(nz, ny, nx, h=h, nshots=nshots, freqs=freqs, nlayers=4, seed=3)
    src = list(true.src)
    # surface receivers, the far corner, an edge node, and one repeated node
    rec = [(0, y, x) for y in range(0, ny, 4) for x in range(0, nx, 4)]
    rec += [(nz - 1, ny - 1, nx - 1), (nz // 2, 0, nx - 1), (0, 4, 8)]
    flat = lambda z, y, x: (z * ny + y) * nx + x
    sv = og.Survey(shape, h, true.freqs, 0.02, [flat(*s) for s in src], [flat(*r) for r in rec])
    d_obs = og.data(true.m, sv)
    return true, start, src, rec, sv, d_obs


def _ctx(hz, m, h):
    import torch
    c = hz.Context(0)
    c.set_model(torch.from_numpy(m), h)
    return c


def test_3d_misfit_matches_oracle(hz):
    import torch
    true, start, src, rec, sv, d_obs = _survey()
    lam = 1e-3
    c = _ctx(hz, start.m, start.h)
    J, d_cal, info = c.misfit_3d(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), lam, tol=1e-11)
    assert len(info) == len(sv.freqs) * len(src)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    J_o = og.misfit(start.m, sv, d_obs, lam)
    assert abs(J - J_o) <= 1e-8 * J_o
    d_o = og.data(start.m, sv)
    assert np.linalg.norm(d_cal.cpu().numpy() - d_o) <= 1e-8 * np.linalg.norm(d_o)


def test_3d_gradient_matches_oracle(hz):
    import torch
    true, start, src, rec, sv, d_obs = _survey()
    lam = 1e-3
    J_o, g_o = og.gradient(start.m, sv, d_obs, lam)
    c = _ctx(hz, start.m, start.h)
    J, g, info = c.gradient_3d(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), lam, tol=1e-11)
    assert len(info) == 2 * len(sv.freqs) * len(src)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    assert abs(J - J_o) <= 1e-8 * J_o
    g = g.cpu().numpy()
    assert g.shape == start.shape
    assert np.linalg.norm(g - g_o) <= 1e-6 * np.linalg.norm(g_o)
    # boundary planes, edges and corners carry the absorbing term's derivative
    for sl in (np.s_[0], np.s_[:, 0], np.s_[:, :, -1], np.s_[0, 0], np.s_[-1, -1, -1]):
        assert np.linalg.norm(g[sl] - g_o[sl]) <= 1e-6 * np.linalg.norm(g_o), sl


def test_3d_gradient_finite_difference_on_gpu_misfit(hz):
    import torch
    true, start, src, rec, sv, d_obs = _survey(shape=(9, 11, 13), nshots=2, freqs=(2.5,))
    lam = 1e-3
    c = _ctx(hz, start.m, start.h)
    dobs_t = torch.from_numpy(d_obs)
    J, g, _ = c.gradient_3d(sv.freqs, sv.alpha, src, rec, dobs_t, lam, tol=1e-12)
    g = g.cpu().numpy()
    Z, Y, X = np.meshgrid(*(np.linspace(0, 1, n) for n in start.shape), indexing="ij")
    v = np.cos(np.pi * X + 0.3) * np.cos(2 * np.pi * Y) * (1 + Z) * np.abs(start.m).max()
    eps = 1e-4
    Js = []
    for sgn in (1.0, -1.0):
        c.set_model(torch.from_numpy(start.m + sgn * eps * v), start.h)
        Jp, _, _ = c.misfit_3d(sv.freqs, sv.alpha, src, rec, dobs_t, lam, tol=1e-12)
        Js.append(Jp)
    fd = (Js[0] - Js[1]) / (2 * eps)
    an = float(np.sum(g * v))
    assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


@pytest.mark.parametrize("cg_iters", [1, 3])
def test_3d_gauss_newton_step_matches_oracle(hz, cg_iters):
    import torch
    true, start, src, rec, sv, d_obs = _survey(shape=(9, 11, 13), nshots=2, freqs=(2.0, 3.0))
    lam = 1e-4
    _, dm_o, J_o, it_o = og.gauss_newton_step(start.m, sv, d_obs, lam, cg_iters=cg_iters)
    c = _ctx(hz, start.m, start.h)
    dm, J, it, info = c.gn_step_3d(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), lam, cg_iters,
                                   tol=1e-12)
    assert it == it_o == cg_iters
    assert abs(J - J_o) <= 1e-9 * J_o
    dm = dm.cpu().numpy()
    assert dm.shape == start.shape
    assert np.linalg.norm(dm - dm_o) <= 1e-6 * np.linalg.norm(dm_o)
    assert og.misfit(start.m + 1e-2 * dm, sv, d_obs, lam) < J_o


def test_3d_fwi_refusals(hz):
    """The 3D calls refuse a 2D model and points outside the box or given
    with two indices; the 2D calls refuse a 3D model."""
    import torch
    w = workloads.model_3d_layered(9, 9, 9, h=30.0, nshots=1, freqs=(3.0,))
    c = _ctx(hz, w.m, w.h)
    d_obs = torch.zeros((1, 1, 1), dtype=torch.complex128)
    for call in (c.gradient, c.misfit):
        with pytest.raises(hz.HzError) as e:
            call(w.freqs, w.alpha, [(0, 4)], [(0, 5)], d_obs, 0.0)
        assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.gn_step(w.freqs, w.alpha, [(0, 4)], [(0, 5)], d_obs, 0.0, 1)
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.gradient_3d(w.freqs, w.alpha, [(0, 4, 4)], [(0, 9, 5)], d_obs, 0.0)
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c.misfit_3d(w.freqs, w.alpha, [(-1, 4, 4)], [(0, 2, 5)], d_obs, 0.0)
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(ValueError):
        c.misfit_3d(w.freqs, w.alpha, [(0, 4)], [(0, 2, 5)], d_obs, 0.0)
    c2 = _ctx(hz, np.full((9, 9), 1 / 2000.0), 30.0)
    with pytest.raises(hz.HzError) as e:
        c2.gradient_3d(w.freqs, w.alpha, [(0, 1, 1)], [(0, 1, 2)], d_obs, 0.0)
    assert e.value.code == hz.HZ_ERR_ARG
    with pytest.raises(hz.HzError) as e:
        c2.gn_step_3d(w.freqs, w.alpha, [(0, 1, 1)], [(0, 1, 2)], d_obs, 0.0, 1)
    assert e.value.code == hz.HZ_ERR_ARG


def test_3d_autograd_function(hz):
    import torch
    true, start, src, rec, sv, d_obs = _survey(shape=(9, 11, 13), nshots=2, freqs=(2.5,))
    c = _ctx(hz, start.m, start.h)
    f = hz.Misfit(c, sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), 1e-3, tol=1e-11)
    m = torch.from_numpy(start.m).cuda().requires_grad_(True)
    J = f(m)
    J.backward()
    J2, g2, _ = c.gradient_3d(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), 1e-3, tol=1e-11)
    assert abs(J.item() - J2) <= 1e-12 * J2
    assert torch.equal(m.grad, g2)


def test_3d_chunked_gradient_matches_full(hz):
    """A workspace budget that admits one frequency at a time gives the same
    3D gradient (forward fields recomputed per chunk)."""
    import torch
    true, start, src, rec, sv, d_obs = _survey(shape=(9, 11, 13), nshots=3, freqs=(2.0, 3.0, 4.0))
    c = _ctx(hz, start.m, start.h)
    # 15 complex vectors per right-hand side and frequency: 720 bytes per node for three shots;
    # three levels keep the dense coarsest level (3 x 3 x 4) inside the budget
    J, g, _ = c.gradient_3d(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), 1e-3, tol=1e-11, levels=3)
    c2 = hz.Context(0, budget_bytes=1000 * start.m.size)
    c2.set_model(torch.from_numpy(start.m), start.h)
    J2, g2, info2 = c2.gradient_3d(sv.freqs, sv.alpha, src, rec, torch.from_numpy(d_obs), 1e-3, tol=1e-11,
                                   levels=3)
    assert len(info2) == 2 * len(sv.freqs) * len(src)
    assert abs(J - J2) <= 1e-10 * J
    assert torch.allclose(g, g2, rtol=0, atol=1e-8 * float(g.abs().max()))
