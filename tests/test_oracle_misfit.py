"""Pins of the misfit J(m) of Eq. (4) against a brute-force triple loop over
frequencies, shots and receivers, and of receiver sampling against direct
indexing."""

import numpy as np

from oracle import misfit


def test_misfit_brute_force():
    rng = np.random.default_rng(4)
    nf, ns, nr = 3, 4, 5
    d_obs = rng.standard_normal((nf, ns, nr)) + 1j * rng.standard_normal((nf, ns, nr))
    d_cal = rng.standard_normal((nf, ns, nr)) + 1j * rng.standard_normal((nf, ns, nr))
    m = rng.uniform(1 / 3000, 1 / 1500, size=(6, 7))
    lam = 1e-3
    J = 0.0
    for f in range(nf):
        for s in range(ns):
            for r in range(nr):
                J += abs(d_obs[f, s, r] - d_cal[f, s, r]) ** 2
    for v in m.ravel():
        J += lam * v * v
    assert np.isclose(misfit.misfit(d_obs, d_cal, m, lam), J, rtol=1e-14, atol=0)
    assert misfit.misfit(d_obs, d_obs, m, lam) == lam * float(np.sum(m ** 2))


def test_sampling_picks_receiver_nodes():
    u = np.arange(2 * 3 * 20).reshape(2, 3, 20) * (1 + 2j)
    rec = [0, 7, 19]
    d = misfit.sample(u, rec)
    assert d.shape == (2, 3, 3)
    assert np.array_equal(d[1, 2], u[1, 2, rec])
