"""The allocation-free solve (hz_solve_noalloc, workspace in the library's
static device array) against hz_solve on the same inputs: two calls in a
row, the second with a smaller batch, each bitwise equal to hz_solve (the
same kernels and reductions; results do not depend on the launch shape),
the context's own workspace untouched by them, and a batch whose workspace
exceeds the array refused before any device work."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import direct
import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("krylov", ["bicgstab", "gmres"])
def test_noalloc_solve_matches_solve(hz, krylov):
    import torch
    w = workloads.model_2d_layered(nz=65, nx=129, h=40.0, nshots=3, freqs=(3.0, 5.0))
    c = hz.Context(0)
    c.set_model(torch.from_numpy(w.m).cuda(), w.h)
    ns = len(w.src)
    b1 = c.point_rhs([0] * ns, w.src)
    cases = [(list(w.freqs), torch.stack([b1] * len(w.freqs))),    # 2 frequencies x 3 shots
             ([w.freqs[1]], b1[:2].reshape((1, 2) + w.shape).contiguous())]  # then 1 x 2: smaller
    refs = []
    for freqs, b in cases:
        print(f"case {len(freqs)} x {b.shape[1]} on {w.shape}", flush=True)
        u_ref, info_ref = c.solve(freqs, w.alpha, b, tol=1e-10, krylov=krylov)
        refs.append((u_ref.clone(), info_ref))
    for (freqs, b), (u_ref, info_ref) in zip(cases, refs):
        out = torch.full_like(b, complex(float("nan"), float("nan")))
        u, info = c.solve(freqs, w.alpha, b, out=out, noalloc=True, tol=1e-10, krylov=krylov)
        assert u.data_ptr() == out.data_ptr()
        assert all(i[0] == hz.HZ_RHS_CONVERGED for i in info), info
        assert [i[1] for i in info] == [i[1] for i in info_ref]
        assert torch.equal(u, u_ref)
    # against the oracle's direct solve (the last, smaller case)
    B = op.operator_B(w.m, w.h, 2 * np.pi * w.freqs[1], w.alpha)
    for s in range(2):
        ref = direct.solve_superlu(B, op.point_source(w.shape, w.h, [w.src[s]]))
        assert rel(u[0, s].cpu().numpy().ravel(), ref) < 1e-8
    # the context's own workspace and coarse inverses are intact
    u2, info2 = c.solve(cases[0][0], w.alpha, cases[0][1], tol=1e-10, krylov=krylov)
    assert torch.equal(u2, refs[0][0])


def test_noalloc_refuses_a_workspace_above_the_array(hz):
    import torch
    w = workloads.model_2d_layered(nz=257, nx=257, h=20.0, nshots=32, freqs=(3.0,))
    c = hz.Context(0)
    c.set_model(torch.from_numpy(w.m).cuda(), w.h)
    b = c.point_rhs([0] * len(w.src), w.src)[None]
    out = torch.empty_like(b)
    assert hz.footprint(w.shape, 1, len(w.src)) > (64 << 20)
    with pytest.raises(hz.HzError) as ei:
        c.solve(list(w.freqs), w.alpha, b, out=out, noalloc=True)
    assert ei.value.code == hz.HZ_ERR_NOMEM and "allocation-free" in str(ei.value)
    # a batch that fits still runs on the same context
    u, info = c.solve(list(w.freqs), w.alpha, b[:, :1].contiguous(), noalloc=True, tol=1e-8)
    assert info[0][0] == hz.HZ_RHS_CONVERGED
