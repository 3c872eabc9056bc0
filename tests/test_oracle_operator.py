"""Pins of the oracle's operator, sources and direct solves against what the
mathematics fixes: exact symmetry, the Neumann null space, the exact discrete
1D solution, the continuum 1D solutions (homogeneous and three layers), a 2D
manufactured solution, the 2D free-space Green's function, reciprocity, and
three independent direct solvers."""

import numpy as np
import pytest
from scipy.special import hankel2

from oracle import operator as op
from oracle import direct


def test_symmetric_and_neumann():
    rng = np.random.default_rng(1)
    for shape in [(7,), (5, 9), (9, 5), (4, 4)]:
        m = 1 / rng.uniform(1500, 3000, size=shape)
        B = op.operator_B(m, 7.0, 2 * np.pi * 9.0, 0.03)
        assert abs(B - B.T).max() == 0.0
        L, g, w = op.stencil_parts(shape)
        assert np.all(L @ np.ones(L.shape[0]) == 0.0)
        # boundary weight is one on every boundary node, zero inside
        gg = g.reshape(shape)
        inner = gg[1:-1] if len(shape) == 1 else gg[1:-1, 1:-1]
        assert np.all(inner == 0)
        assert np.all(np.sort(np.unique(gg)) == np.array([0.0, 1.0]))
        # mass weights sum to the measure of the domain in cell units
        assert np.isclose(w.sum(), np.prod([n - 1 for n in shape]))


def test_interior_rows_are_textbook_helmholtz():
    """Away from the boundary, a row is (4u - sum of neighbours)/h^2 - k^2(1-j alpha) u."""
    nz, nx, h, om, al = 6, 7, 3.0, 11.0, 0.2
    m = np.full((nz, nx), 1 / 2000.0)
    B = op.operator_B(m, h, om, al).toarray()
    p = 2 * nx + 3
    row = B[p]
    assert np.isclose(row[p], 4 / h ** 2 - om ** 2 * m[0, 0] ** 2 * (1 - 1j * al))
    for q in (p - 1, p + 1, p - nx, p + nx):
        assert row[q] == -1 / h ** 2
    assert np.count_nonzero(row) == 5


def _discrete_1d_closed_form(n, h, k, kappa2, src_amp):
    """Homogeneous 1D: interior rows force u_i = A z^i + C z^-i with
    2 - 2 cos(theta) = kappa^2 h^2, z = exp(-j theta). The two end rows come
    from the unweighted three-point stencil with the ghost node eliminated by
    the centred condition -u'(0) + j k u(0) = 0 (left) and
    u'(L) + j k u(L) = 0 (right), each multiplied by its half weight."""
    theta = np.arccos(1 - kappa2 * h ** 2 / 2 + 0j)
    z = np.exp(-1j * theta)
    i = np.arange(n)

    def end_row(u_end, u_next):
        ghost = u_next - 2j * k * h * u_end
        return 0.5 * ((-ghost + 2 * u_end - u_next) / h ** 2 - kappa2 * u_end)

    # left row as a linear function of (A, C)
    la = end_row(1.0, z)
    lc = end_row(1.0, 1 / z)
    ra = end_row(z ** (n - 1), z ** (n - 2))
    rc = end_row(z ** -(n - 1), z ** -(n - 2))
    A, C = np.linalg.solve(np.array([[la, lc], [ra, rc]]), np.array([src_amp, 0.0]))
    return A * z ** i + C * z ** (-i)


def test_1d_exact_discrete_solution():
    n, h, f, al, c = 301, 5.0, 10.0, 0.01, 1500.0
    om = 2 * np.pi * f
    m = np.full(n, 1 / c)
    B = op.operator_B(m, h, om, al)
    b = op.point_source((n,), h, [0])
    u = direct.solve_superlu(B, b)
    k = om / c
    ref = _discrete_1d_closed_form(n, h, k, k ** 2 * (1 - 1j * al), 1 / h)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-11


def _continuum_1d(x, L, k, kappa):
    """-u'' - kappa^2 u = 0 on (0, L); -u'(0) + j k u(0) = 1; u'(L) + j k u(L) = 0."""
    E = np.exp(-2j * kappa * L)
    A = 1 / (1j * (kappa + k) - 1j * (k - kappa) ** 2 * E / (k + kappa))
    Bc = -(k - kappa) / (k + kappa) * A * E
    return A * np.exp(-1j * kappa * x) + Bc * np.exp(1j * kappa * x)


def test_1d_continuum_second_order():
    L, f, al, c = 5000.0, 10.0, 0.01, 1500.0
    om = 2 * np.pi * f
    k = om / c
    kappa = k * np.sqrt(1 - 1j * al)
    errs = []
    for n in (1001, 2001, 4001):
        h = L / (n - 1)
        x = np.arange(n) * h
        u = direct.solve_superlu(op.operator_B(np.full(n, 1 / c), h, om, al),
                                 op.point_source((n,), h, [0]))
        ref = _continuum_1d(x, L, k, kappa)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.9 < r1 < 4.1 and 3.9 < r2 < 4.1, errs
    assert 0.15 < errs[0] < 0.18  # 1001 nodes at 10 Hz: about 15 points per damped wavelength


def _continuum_1d_layers(x, edges, cs, om, al):
    """Piecewise A_l e^{-j kappa_l x} + C_l e^{j kappa_l x}, u and u' continuous at
    the interfaces, source condition at x = 0 and absorbing end at x = L."""
    nl = len(cs)
    ks = [om / c for c in cs]
    kap = [kk * np.sqrt(1 - 1j * al) for kk in ks]
    M = np.zeros((2 * nl, 2 * nl), dtype=complex)
    r = np.zeros(2 * nl, dtype=complex)
    # left: -u'(0) + j k0 u(0) = 1
    M[0, 0] = 1j * kap[0] + 1j * ks[0]
    M[0, 1] = -1j * kap[0] + 1j * ks[0]
    r[0] = 1.0
    row = 1
    for l in range(nl - 1):
        xi = edges[l]
        ea, ec = np.exp(-1j * kap[l] * xi), np.exp(1j * kap[l] * xi)
        fa, fc = np.exp(-1j * kap[l + 1] * xi), np.exp(1j * kap[l + 1] * xi)
        M[row, 2 * l:2 * l + 2] = [ea, ec]
        M[row, 2 * l + 2:2 * l + 4] = [-fa, -fc]
        M[row + 1, 2 * l:2 * l + 2] = [-1j * kap[l] * ea, 1j * kap[l] * ec]
        M[row + 1, 2 * l + 2:2 * l + 4] = [1j * kap[l + 1] * fa, -1j * kap[l + 1] * fc]
        row += 2
    xl = x[-1]
    kk, ka = ks[-1], kap[-1]
    M[row, -2] = (-1j * ka + 1j * kk) * np.exp(-1j * ka * xl)
    M[row, -1] = (1j * ka + 1j * kk) * np.exp(1j * ka * xl)
    coef = np.linalg.solve(M, r)
    u = np.zeros(len(x), dtype=complex)
    bounds = [0.0] + list(edges) + [np.inf]
    for l in range(nl):
        sel = (x >= bounds[l]) & (x < bounds[l + 1]) if l < nl - 1 else (x >= bounds[l])
        u[sel] = coef[2 * l] * np.exp(-1j * kap[l] * x[sel]) + coef[2 * l + 1] * np.exp(1j * kap[l] * x[sel])
    return u


def test_1d_three_layers_converges_second_order():
    """Interfaces on nodes carrying the mean squared slowness of both sides."""
    Ltot, f, al = 4800.0, 5.0, 0.01
    cs = [1500.0, 2200.0, 3000.0]
    edges = [1600.0, 3200.0]
    om = 2 * np.pi * f
    errs = []
    for n in (601, 1201, 2401):
        h = Ltot / (n - 1)
        x = np.arange(n) * h
        m = np.where(x < edges[0], 1 / cs[0], np.where(x < edges[1], 1 / cs[1], 1 / cs[2]))
        for e, (ca, cb) in zip(edges, [(cs[0], cs[1]), (cs[1], cs[2])]):
            i = int(round(e / h))
            m[i] = np.sqrt(0.5 * (1 / ca ** 2 + 1 / cb ** 2))
        u = direct.solve_superlu(op.operator_B(m, h, om, al), op.point_source((n,), h, [0]))
        ref = _continuum_1d_layers(x, edges, cs, om, al)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def _manufactured_2d(n, Lx, Lz, c, om, al):
    """u* = cos(pi x/Lx) cos(pi z/Lz) exp(-j k0 x): returns (u*, weighted rhs).

    The rhs is W f plus the absorbing-boundary data g = du*/dn + j k u*: a
    ghost node beyond an edge is u_inner - 2 j k h u_b + 2 h g, so each end
    direction adds (weight of the other axis) * g / h to the row."""
    nx, nz = n
    hx = Lx / (nx - 1)
    h = hx
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    Z, X = np.meshgrid(z, x, indexing="ij")
    k = om / c
    k0 = 0.7 * k
    ax, az = np.pi / Lx, np.pi / Lz
    cxs, sxs = np.cos(ax * X), np.sin(ax * X)
    czs, szs = np.cos(az * Z), np.sin(az * Z)
    ph = np.exp(-1j * k0 * X)
    u = cxs * czs * ph
    ux = (-ax * sxs - 1j * k0 * cxs) * czs * ph
    uz = -az * cxs * szs * ph
    uxx = (-ax ** 2 * cxs + 2j * k0 * ax * sxs - k0 ** 2 * cxs) * czs * ph
    uzz = -az ** 2 * u
    kap2 = k ** 2 * (1 - 1j * al)
    f = -(uxx + uzz) - kap2 * u
    wz = op.end_weights(nz)
    wx = op.end_weights(nx)
    b = np.outer(wz, wx) * f
    # outward normals: -x at ix=0, +x at ix=nx-1, -z at iz=0, +z at iz=nz-1
    b[:, 0] += wz * (-ux[:, 0] + 1j * k * u[:, 0]) / h
    b[:, -1] += wz * (ux[:, -1] + 1j * k * u[:, -1]) / h
    b[0, :] += wx * (-uz[0, :] + 1j * k * u[0, :]) / h
    b[-1, :] += wx * (uz[-1, :] + 1j * k * u[-1, :]) / h
    return u.ravel(), b.ravel(), h


def test_2d_manufactured_second_order():
    Lx, Lz, c, f, al = 1200.0, 800.0, 2000.0, 4.0, 0.05
    om = 2 * np.pi * f
    errs = []
    for nx in (61, 121, 241):
        nz = (nx - 1) * 2 // 3 + 1
        u, b, h = _manufactured_2d((nx, nz), Lx, Lz, c, om, al)
        B = op.operator_B(np.full((nz, nx), 1 / c), h, om, al)
        x = direct.solve_superlu(B, b)
        errs.append(np.linalg.norm(x - u) / np.linalg.norm(u))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_2d_point_source_matches_free_space_green():
    """Centre source in a damped homogeneous square: near the source (a few
    wavelengths, far from the edges) u ~ -(j/4) H0^(2)(kappa r)."""
    n, h, c, f, al = 241, 5.0, 2000.0, 10.0, 0.1
    om = 2 * np.pi * f
    kap = om / c * np.sqrt(1 - 1j * al)
    m = np.full((n, n), 1 / c)
    s = (n // 2) * n + n // 2
    u = direct.solve_superlu(op.operator_B(m, h, om, al), op.point_source((n, n), h, [s]))
    u = u.reshape(n, n)
    ic = n // 2
    for d in (20, 30, 40):  # 0.5 .. 1 wavelength (200 m) away, along an axis and a diagonal
        for (iz, ix) in ((ic, ic + d), (ic + d, ic)):
            r = d * h
            ref = -0.25j * hankel2(0, kap * r)
            assert abs(u[iz, ix] - ref) / abs(ref) < 0.02
        dd = int(round(d / np.sqrt(2)))
        r = dd * h * np.sqrt(2)
        ref = -0.25j * hankel2(0, kap * r)
        assert abs(u[ic + dd, ic + dd] - ref) / abs(ref) < 0.02


def test_reciprocity_with_surface_nodes():
    rng = np.random.default_rng(3)
    shape, h = (41, 61), 10.0
    m = 1 / rng.uniform(1500, 2500, size=shape)
    B = op.operator_B(m, h, 2 * np.pi * 6.0, 0.01)
    s, r = 17, 20 * 61 + 45  # a surface node and an interior node
    us = direct.solve_superlu(B, op.point_source(shape, h, [s]))
    ur = direct.solve_superlu(B, op.point_source(shape, h, [r]))
    assert abs(us[r] - ur[s]) <= 1e-12 * abs(us[r])
    s2, r2 = 0, 60  # two surface corners
    u1 = direct.solve_superlu(B, op.point_source(shape, h, [s2]))
    u2 = direct.solve_superlu(B, op.point_source(shape, h, [r2]))
    assert abs(u1[r2] - u2[s2]) <= 1e-12 * abs(u1[r2])


@pytest.mark.parametrize("shape", [(33,), (9, 13), (13, 9), (17, 17)])
def test_three_direct_solvers_agree(shape):
    rng = np.random.default_rng(7)
    m = 1 / rng.uniform(1500, 3000, size=shape)
    B = op.operator_B(m, 10.0, 2 * np.pi * 15.0, 0.01)
    b = rng.standard_normal(B.shape[0]) + 1j * rng.standard_normal(B.shape[0])
    x1 = direct.solve_superlu(B, b)
    x2 = direct.solve_dense(B, b)
    x3 = direct.solve_banded(B, b, shape)
    for x in (x1, x3):
        assert np.linalg.norm(x - x2) <= 1e-12 * np.linalg.norm(x2)
    assert np.linalg.norm(B @ x3 - b) <= 1e-12 * np.linalg.norm(b) * np.abs(B).max() * 10


def test_discrete_manufactured_solution_recovered():
    rng = np.random.default_rng(11)
    shape = (31, 45)
    m = 1 / rng.uniform(1500, 3000, size=shape)
    B = op.operator_B(m, 10.0, 2 * np.pi * 8.0, 0.01)
    ustar = rng.standard_normal(B.shape[0]) + 1j * rng.standard_normal(B.shape[0])
    u = direct.solve_superlu(B, B @ ustar)
    assert np.linalg.norm(u - ustar) <= 1e-11 * np.linalg.norm(ustar)


def test_point_source_scaling():
    b1 = op.point_source((9,), 4.0, [0, 3], [1.0, 2.0 + 1j])
    assert b1[0] == 0.25 and b1[3] == (2.0 + 1j) / 4.0
    b2 = op.point_source((5, 7), 4.0, [8])
    assert b2[8] == 1 / 16.0 and np.count_nonzero(b2) == 1
