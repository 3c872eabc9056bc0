"""GPU checks of the FWI pieces at the full size of the Gauss-Newton
configuration: 301 x 601, 32 surface shots, 151 surface receivers,
3/4/6/8/10/12 Hz, lambda = 1e-3, observed data from the oracle's direct
solves on the true model (as the paper generates its observed data).

* the gradient of a sampled sub-survey (two shots at two frequencies)
  against the oracle's gradient (direct solves), 1e-6 relative;
* the gradient of the whole survey against central differences of the GPU
  misfit along a smooth direction (a property that holds at any size), and
  the autograd wrapper against it;
* one Gauss-Newton step of the whole survey is a descent direction that
  lowers J.
"""

import numpy as np
import pytest

from oracle import gradient as og
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def survey():
    w = workloads.model_fwi()
    nx = w.shape[1]
    sv = og.Survey(w.shape, w.h, w.freqs, w.alpha, list(w.src), [ix for ix in w.rec])
    print(f"[fwi-full] oracle observed data: {len(w.freqs)} frequencies x {len(w.src)} shots", flush=True)
    d_obs = og.data(w.m, sv)
    src = [(0, ix) for ix in w.src]
    rec = [(0, ix) for ix in w.rec]
    assert all(0 <= ix < nx for ix in w.rec)
    return w, sv, d_obs, src, rec


def _ctx(hz, m, h):
    import torch
    c = hz.Context(0)
    c.set_model(torch.from_numpy(np.ascontiguousarray(m)), h)
    return c


def test_subsurvey_gradient_matches_oracle(hz, survey):
    import torch
    w, sv, d_obs, src, rec = survey
    shots, fidx = [0, 31], [0, 3]
    sub = og.Survey(w.shape, w.h, [w.freqs[i] for i in fidx], w.alpha, [w.src[s] for s in shots], list(w.rec))
    d_sub = d_obs[np.ix_(fidx, shots)]
    J_o, g_o = og.gradient(w.m_start, sub, d_sub, w.lam)
    c = _ctx(hz, w.m_start, w.h)
    J, g, info = c.gradient(sub.freqs, w.alpha, [src[s] for s in shots], rec, torch.from_numpy(d_sub), w.lam,
                            tol=1e-11)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    assert abs(J - J_o) <= 1e-8 * J_o
    g = g.cpu().numpy()
    assert np.linalg.norm(g - g_o) <= 1e-6 * np.linalg.norm(g_o)


def test_full_survey_gradient_finite_difference_and_autograd(hz, survey):
    import torch
    w, sv, d_obs, src, rec = survey
    dobs_t = torch.from_numpy(d_obs)
    c = _ctx(hz, w.m_start, w.h)
    J, g, info = c.gradient(w.freqs, w.alpha, src, rec, dobs_t, w.lam, tol=1e-11)
    assert len(info) == 2 * len(w.freqs) * len(w.src)
    assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info)
    v = workloads.smooth_random_vectors(1, w.shape, 11, sigma=8.0)[0].real.reshape(w.shape)
    v = v / np.abs(v).max() * np.abs(w.m_start).max()
    eps = 1e-4
    Js = []
    for sgn in (1.0, -1.0):
        c.set_model(torch.from_numpy(w.m_start + sgn * eps * v), w.h)
        Jp, _, _ = c.misfit(w.freqs, w.alpha, src, rec, dobs_t, w.lam, tol=1e-11)
        Js.append(Jp)
    fd = (Js[0] - Js[1]) / (2 * eps)
    an = float(np.sum(g.cpu().numpy() * v))
    assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)
    c.set_model(torch.from_numpy(w.m_start), w.h)
    f = hz.Misfit(c, w.freqs, w.alpha, src, rec, dobs_t, w.lam, tol=1e-11)
    m = torch.from_numpy(w.m_start).cuda().requires_grad_(True)
    Jt = f(m)
    Jt.backward()
    assert abs(Jt.item() - J) <= 1e-12 * J
    assert torch.equal(m.grad, g)


def test_full_survey_gauss_newton_step_descends(hz, survey):
    import torch
    w, sv, d_obs, src, rec = survey
    dobs_t = torch.from_numpy(d_obs)
    c = _ctx(hz, w.m_start, w.h)
    J0, g, _ = c.gradient(w.freqs, w.alpha, src, rec, dobs_t, w.lam, tol=1e-10)
    dm, J, it, info = c.gn_step(w.freqs, w.alpha, src, rec, dobs_t, w.lam, 3, tol=1e-10)
    assert it == 3
    assert abs(J - J0) <= 1e-9 * J0
    dm = dm.cpu().numpy()
    assert float(np.sum(g.cpu().numpy() * dm)) < 0.0
    c.set_model(torch.from_numpy(w.m_start + 0.25 * dm), w.h)
    J1, _, _ = c.misfit(w.freqs, w.alpha, src, rec, dobs_t, w.lam, tol=1e-10)
    assert J1 < J0
