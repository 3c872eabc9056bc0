"""Pins of the oracle on 3D grids (Eq. (1) with d = 3, constant density as in
Eq. (2)): the operator, the multigrid transfers, the V-cycle and the local
Fourier analysis, each against something other than the oracle itself --
exact algebraic properties, closed-form weight sums, the textbook 7-point
stencil, a manufactured continuum solution (second order), the free-space
Green's function, trilinear functions, the explicit error-propagation matrix
and a brute-force Fourier sweep."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
from oracle import lfa
from oracle import direct


def test_3d_symmetric_neumann_and_weight_sums():
    rng = np.random.default_rng(11)
    for shape in [(5, 6, 7), (4, 4, 4), (3, 5, 4)]:
        m = 1 / rng.uniform(1500, 3000, size=shape)
        B = op.operator_B(m, 7.0, 2 * np.pi * 9.0, 0.03)
        assert abs(B - B.T).max() == 0.0
        L, g, w = op.stencil_parts(shape)
        assert np.all(L @ np.ones(L.shape[0]) == 0.0)
        nz, ny, nx = (n - 1 for n in shape)
        # mass weights: the box's volume; boundary weights: its surface, in cell units
        assert w.sum() == nz * ny * nx
        assert g.sum() == 2 * (nz * ny + ny * nx + nz * nx)
        gg = g.reshape(shape)
        assert np.all(gg[1:-1, 1:-1, 1:-1] == 0)
        # a corner node exposes three quarter faces, every other boundary node one full face
        assert gg[0, 0, 0] == 0.75 and gg[-1, -1, -1] == 0.75
        assert np.all(np.isin(np.unique(gg), [0.0, 0.75, 1.0]))


def test_3d_interior_rows_are_textbook_helmholtz():
    """Away from the boundary, a row is (6u - sum of the six neighbours)/h^2 - k^2(1-j alpha) u."""
    nz, ny, nx, h, om, al = 5, 6, 7, 3.0, 11.0, 0.2
    m = np.full((nz, ny, nx), 1 / 2000.0)
    B = op.operator_B(m, h, om, al).tocsr()
    p = (2 * ny + 3) * nx + 3
    row = B[p].toarray().ravel()
    assert np.isclose(row[p], 6 / h ** 2 - om ** 2 * m[0, 0, 0] ** 2 * (1 - 1j * al))
    for q in (p - 1, p + 1, p - nx, p + nx, p - nx * ny, p + nx * ny):
        assert row[q] == -1 / h ** 2
    assert np.count_nonzero(row) == 7


def _manufactured_3d(shape, lengths, c, om, al):
    """u* = cos(pi x/Lx) cos(pi y/Ly) cos(pi z/Lz) exp(-j k0 x): returns
    (u*, weighted rhs, h). The rhs is W f plus the absorbing-boundary data
    g = du*/dn + j k u* on every face, each end direction adding the face's
    weight (the product of the other two axes' weights) times g / h."""
    nz, ny, nx = shape
    Lz, Ly, Lx = lengths
    h = Lx / (nx - 1)
    assert np.isclose(Ly / (ny - 1), h) and np.isclose(Lz / (nz - 1), h)
    z, y, x = (np.arange(n) * h for n in shape)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    k = om / c
    k0 = 0.7 * k
    ax, ay, az = np.pi / Lx, np.pi / Ly, np.pi / Lz
    cx, sx = np.cos(ax * X), np.sin(ax * X)
    cy, sy = np.cos(ay * Y), np.sin(ay * Y)
    cz, sz = np.cos(az * Z), np.sin(az * Z)
    ph = np.exp(-1j * k0 * X)
    u = cx * cy * cz * ph
    ux = (-ax * sx - 1j * k0 * cx) * cy * cz * ph
    uy = -ay * cx * sy * cz * ph
    uz = -az * cx * cy * sz * ph
    uxx = (-ax ** 2 * cx + 2j * k0 * ax * sx - k0 ** 2 * cx) * cy * cz * ph
    lap = uxx - ay ** 2 * u - az ** 2 * u
    f = -lap - k ** 2 * (1 - 1j * al) * u
    wz, wy, wx = (op.end_weights(n) for n in shape)
    b = wz[:, None, None] * wy[None, :, None] * wx[None, None, :] * f
    fx = wz[:, None] * wy[None, :]   # face weight of the x-faces, over (z, y)
    fy = wz[:, None] * wx[None, :]   # y-faces, over (z, x)
    fz = wy[:, None] * wx[None, :]   # z-faces, over (y, x)
    b[:, :, 0] += fx * (-ux[:, :, 0] + 1j * k * u[:, :, 0]) / h
    b[:, :, -1] += fx * (ux[:, :, -1] + 1j * k * u[:, :, -1]) / h
    b[:, 0, :] += fy * (-uy[:, 0, :] + 1j * k * u[:, 0, :]) / h
    b[:, -1, :] += fy * (uy[:, -1, :] + 1j * k * u[:, -1, :]) / h
    b[0, :, :] += fz * (-uz[0, :, :] + 1j * k * u[0, :, :]) / h
    b[-1, :, :] += fz * (uz[-1, :, :] + 1j * k * u[-1, :, :]) / h
    return u.ravel(), b.ravel(), h


def test_3d_manufactured_second_order():
    lengths, c, f, al = (600.0, 800.0, 1200.0), 2000.0, 1.5, 0.05
    om = 2 * np.pi * f
    errs = []
    for nx in (13, 25, 49):
        shape = ((nx - 1) // 2 + 1, (nx - 1) * 2 // 3 + 1, nx)
        u, b, h = _manufactured_3d(shape, lengths, c, om, al)
        B = op.operator_B(np.full(shape, 1 / c), h, om, al)
        x = direct.solve_superlu(B, b)
        errs.append(np.linalg.norm(x - u) / np.linalg.norm(u))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.6 < r2 < 4.4, errs


def test_3d_point_source_matches_free_space_green():
    """Centre source in a damped homogeneous cube: a few cells away (far
    from the faces) u ~ exp(-j kappa r) / (4 pi r), the outgoing free-space
    Green's function of -Laplace - kappa^2 for the time factor exp(j omega t)."""
    n, h, c, f, al = 33, 5.0, 2000.0, 20.0, 0.3
    om = 2 * np.pi * f
    kap = om / c * np.sqrt(1 - 1j * al)
    m = np.full((n, n, n), 1 / c)
    ic = n // 2
    s = (ic * n + ic) * n + ic
    u = direct.solve_superlu(op.operator_B(m, h, om, al), op.point_source((n, n, n), h, [s]))
    u = u.reshape(n, n, n)
    for d in (4, 6, 8):
        r = d * h
        ref = np.exp(-1j * kap * r) / (4 * np.pi * r)
        for (iz, iy, ix) in ((ic, ic, ic + d), (ic, ic + d, ic), (ic + d, ic, ic)):
            assert abs(u[iz, iy, ix] - ref) / abs(ref) < 0.05, (d, u[iz, iy, ix], ref)
    # the three axes see the same field (the grid and the source are symmetric)
    assert abs(u[ic, ic, ic + 5] - u[ic + 5, ic, ic]) <= 1e-10 * abs(u[ic, ic, ic + 5])


def test_3d_prolongation_reproduces_trilinear_functions():
    for coarse in [(3, 5, 4), (5, 3, 3)]:
        P = mg.prolongation(coarse)
        fine = tuple(2 * (n - 1) + 1 for n in coarse)
        Zc, Yc, Xc = np.meshgrid(*(np.arange(n) * 2.0 for n in coarse), indexing="ij")
        Zf, Yf, Xf = np.meshgrid(*(np.arange(n) * 1.0 for n in fine), indexing="ij")

        def fn(Z, Y, X):
            return 1 + 0.3 * X - 0.7 * Z + 0.2 * Y + 0.1 * X * Z - 0.05 * Y * Z + 0.02 * X * Y * Z

        assert np.allclose(P @ fn(Zc, Yc, Xc).ravel(), fn(Zf, Yf, Xf).ravel(), rtol=0, atol=1e-12)


def test_3d_restriction_preserves_weighted_constants_and_full_weighting():
    for coarse in [(3, 3, 3), (3, 5, 4)]:
        fine = tuple(2 * (n - 1) + 1 for n in coarse)
        _, _, wf = op.stencil_parts(fine)
        _, _, wc = op.stencil_parts(coarse)
        R = mg.restriction(coarse)
        assert np.allclose(R @ wf, wc, rtol=0, atol=1e-14)
    # interior full weighting: the tensor product of (1 2 1)/4 along each axis
    R = mg.restriction((5, 5, 5)).toarray()
    row = R[(2 * 5 + 2) * 5 + 2].reshape(9, 9, 9)
    k = np.array([1.0, 2.0, 1.0]) / 4.0
    ref = np.zeros((9, 9, 9))
    ref[3:6, 3:6, 3:6] = k[:, None, None] * k[None, :, None] * k[None, None, :]
    assert np.array_equal(row, ref)


@pytest.mark.parametrize("shape,levels,nu", [((9, 9, 9), 2, (2, 2)), ((9, 9, 9), 3, (1, 1))])
def test_3d_vcycle_equals_explicit_error_propagation(shape, levels, nu):
    rng = np.random.default_rng(7)
    m = 1 / rng.uniform(1500, 3000, size=shape)
    h, om = 40.0, 2 * np.pi * 4.0
    vc = mg.VCycle(m, h, om, 1.0, 0.5, levels, nu[0], nu[1], [0.8, 0.6][:levels - 1])
    C = mg.vcycle_matrix(vc)
    b = rng.standard_normal(C.shape[0]) + 1j * rng.standard_normal(C.shape[0])
    assert np.linalg.norm(vc(b) - C @ b) <= 1e-13 * np.linalg.norm(C @ b)
    Minv = np.linalg.inv(vc.M[0].toarray())
    assert np.linalg.norm(C - Minv) > 1e-6 * np.linalg.norm(Minv)


def test_3d_lfa_closed_form_matches_brute_force():
    for kh in (0.1, 0.6, 1.2, 2.3, 3.5):
        for (b1, b2, w) in ((1, 0.5, 0.8), (1, 1, 0.8), (1, 0.5, 0.4)):
            a = lfa.smoothing_factor(kh, b1, b2, w, 3)
            bf = lfa.smoothing_factor_sampled(kh, b1, b2, w, 3, n=65)
            assert abs(a - bf) < 1e-12, (kh, b1, b2, w, a, bf)


def _survey_3d(shape=(7, 8, 9), h=40.0):
    """A small 3D survey: true and starting layered models, surface shots,
    receivers on the surface plane, the far corner and an edge node."""
    from oracle import gradient as og
    import workloads
    nz, ny, nx = shape
    true = workloads.model_3d_layered(nz, ny, nx, h=h, nshots=2, freqs=(2.0, 3.5), nlayers=3)
    start = workloads.model_3d_layered(nz, ny, nx, h=h, nshots=2, freqs=(2.0, 3.5), nlayers=3, seed=5)
    flat = lambda z, y, x: (z * ny + y) * nx + x
    src = [flat(*s) for s in true.src]
    rec = [flat(0, y, x) for y in range(0, ny, 3) for x in range(0, nx, 3)]
    rec += [flat(nz - 1, ny - 1, nx - 1), flat(3, 0, nx - 1)]
    sv = og.Survey(shape, h, true.freqs, 0.05, src, rec)
    return og, start.m, sv, og.data(true.m, sv)


def _smooth_3d(shape, k):
    Z, Y, X = np.meshgrid(*(np.linspace(0, 1, n) for n in shape), indexing="ij")
    return np.cos(k * np.pi * X + 0.3) * np.cos((k + 1) * np.pi * Y) * (1 + Z)


def test_3d_gradient_matches_central_differences():
    """Eq. (7) on a 3D grid: the directional derivative of J along smooth
    directions, and along single face, edge and corner nodes (whose boundary
    term's dependence on m is the exposed face area 1, 1 and 3/4)."""
    og, m, sv, d_obs = _survey_3d()
    lam = 1e3
    J, g = og.gradient(m, sv, d_obs, lam)
    assert np.isclose(J, og.misfit(m, sv, d_obs, lam), rtol=1e-12)
    for k in (1, 2):
        v = _smooth_3d(m.shape, k) * np.abs(m).max()
        eps = 1e-4
        fd = (og.misfit(m + eps * v, sv, d_obs, lam) - og.misfit(m - eps * v, sv, d_obs, lam)) / (2 * eps)
        an = float(np.sum(g * v))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    J0, g0 = og.gradient(m, sv, d_obs, 0.0)
    nz, ny, nx = m.shape
    for node in ((0, 3, 4), (nz - 1, 0, 5), (0, 0, 0), (nz - 1, ny - 1, nx - 1), (3, 4, 0)):
        v = np.zeros_like(m)
        v[node] = m[node]
        eps = 1e-5
        fd = (og.misfit(m + eps * v, sv, d_obs, 0.0) - og.misfit(m - eps * v, sv, d_obs, 0.0)) / (2 * eps)
        assert abs(fd - g0[node] * v[node]) <= 1e-5 * abs(fd) + 1e-12 * J0, node


def test_3d_taylor_remainder_and_born_data():
    og, m, sv, d_obs = _survey_3d()
    J, g = og.gradient(m, sv, d_obs, 0.0)
    v = _smooth_3d(m.shape, 1) * np.abs(m).max()
    rems = [abs(og.misfit(m + e * v, sv, d_obs, 0.0) - J - e * float(np.sum(g * v))) for e in (4e-3, 2e-3, 1e-3)]
    assert 3.5 < rems[0] / rems[1] < 4.5 and 3.5 < rems[1] / rems[2] < 4.5, rems
    eps = 1e-5
    fd = (og.data(m + eps * v, sv) - og.data(m - eps * v, sv)) / (2 * eps)
    gb = og.born(m, sv, v)
    assert np.linalg.norm(fd - gb) <= 1e-6 * np.linalg.norm(gb)
