"""GPU tests of the continuous-admission solve server: requests of different
grids, dimensions, frequencies and right-hand-side counts run at the same time
on separate streams and give, bit for bit, what a standalone context gives for
the same request (every reduction has a fixed order per right-hand side);
admission keeps the summed resident footprint within the memory budget; a
request larger than the budget is refused at submission."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _requests():
    """(m, h, freqs, b) of a mixed stream: 2D lens, 2D layered, 1D layers."""
    import torch
    out = []
    lens = workloads.model_2d_lens(n=65, h=20.0)
    lay = workloads.model_2d_layered(nz=33, nx=129, h=20.0, nshots=6, freqs=(3.0, 5.0))
    one = workloads.model_1d_layers(n=257, h=8.0)
    rng = np.random.default_rng(11)
    for k, (mdl, freqs, nrhs) in enumerate([(lens, (4.0,), 3), (lay, (3.0, 5.0), 6), (one, (6.0, 9.0), 2),
                                             (lens, (2.5, 6.0), 5), (lay, (4.0,), 1), (one, (12.0,), 4)]):
        shape = mdl.shape
        n = int(np.prod(shape))
        b = np.zeros((len(freqs), nrhs, n), dtype=np.complex128)
        for f in range(len(freqs)):
            for r in range(nrhs):
                b[f, r, rng.integers(0, n)] = 1.0 / mdl.h ** len(shape)
        out.append((mdl.m, mdl.h, freqs, torch.from_numpy(b.reshape((len(freqs), nrhs) + tuple(shape)))))
    return out


def _standalone(hz, reqs, **opt):
    import torch
    res = []
    for m, h, freqs, b in reqs:
        c = hz.Context(0)
        c.set_model(torch.from_numpy(m), h)
        u, info = c.solve(freqs, 0.02, b, **opt)
        res.append((u.clone(), info))
        c.close()
    return res


@pytest.mark.parametrize("slots", [1, 3])
def test_concurrent_requests_match_standalone_bitwise(hz, slots):
    import torch
    reqs = _requests()
    ref = _standalone(hz, reqs, tol=1e-9)
    srv = hz.Server(0, slots=slots)
    try:
        tickets = [srv.submit(torch.from_numpy(m), h, freqs, 0.02, b, tol=1e-9) for m, h, freqs, b in reqs]
        for (u_ref, info_ref), tk in zip(ref, tickets):
            u, info, times = srv.wait(tk)
            assert [i[0] for i in info] == [hz.HZ_RHS_CONVERGED] * len(info)
            assert [i[1] for i in info] == [i[1] for i in info_ref]
            assert torch.equal(u, u_ref)
            assert times[0] >= 0.0 and times[1] > 0.0 and times[2] >= times[1]
        st = srv.stats()
        assert st["queued"] == 0 and st["running"] == 0
        assert 1 <= st["peak_running"] <= slots
    finally:
        srv.close()


def test_budget_admission_and_refusal(hz):
    """With a budget that holds one large request but not two, the large
    requests never run together; small ones fill in beside them; results are
    unchanged; a request above the budget is refused."""
    import torch
    big = workloads.model_2d_layered(nz=65, nx=129, h=20.0, nshots=4, freqs=(3.0,))
    small = workloads.model_2d_lens(n=33, h=40.0)
    n_big = big.m.size
    fp_big = hz.footprint(big.shape, 1, 4)
    fp_small = hz.footprint(small.shape, 1, 2)
    assert fp_small < fp_big
    budget = fp_big + 2 * fp_small
    rng = np.random.default_rng(5)

    def rhs(shape, nrhs, h):
        n = int(np.prod(shape))
        b = np.zeros((1, nrhs, n), dtype=np.complex128)
        for r in range(nrhs):
            b[0, r, rng.integers(0, n)] = 1.0 / h ** 2
        return torch.from_numpy(b.reshape((1, nrhs) + tuple(shape)))

    reqs = []
    for k in range(6):
        if k % 2 == 0:
            reqs.append((big.m, big.h, (3.0 + k,), rhs(big.shape, 4, big.h)))
        else:
            reqs.append((small.m, small.h, (1.5 + 0.5 * k,), rhs(small.shape, 2, small.h)))
    ref = _standalone(hz, reqs, tol=1e-8)
    srv = hz.Server(0, budget_bytes=budget, slots=3)
    try:
        with pytest.raises(hz.HzError) as e:
            srv.submit(torch.from_numpy(big.m), big.h, (3.0,), 0.02, rhs(big.shape, 8, big.h), tol=1e-8)
        assert e.value.code == hz.HZ_ERR_NOMEM
        tickets = [srv.submit(torch.from_numpy(m), h, f, 0.02, b, tol=1e-8) for m, h, f, b in reqs]
        peak_bytes = 0
        for (u_ref, _), tk in zip(ref, tickets):
            peak_bytes = max(peak_bytes, srv.stats()["bytes"])
            u, info, _ = srv.wait(tk)
            assert torch.equal(u, u_ref)
        assert peak_bytes <= budget
        assert n_big > small.m.size
    finally:
        srv.close()
