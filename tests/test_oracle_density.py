"""Pins of the oracle's variable-density operator (Eq. (1)): the constant
density identity, exact symmetry and the Neumann null space, second-order
convergence to manufactured solutions of -div(rho grad u) - k^2 (1 - j alpha) u
= f with the flux absorbing condition in 1D and 2D, the V-cycle's explicit
matrix and its constant-density scaling, the coarse operator against the
Galerkin product, the coarse policy's slowness and the gradient against
finite differences."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
from oracle import direct
from oracle import gradient as og
import workloads


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    m = 1 / rng.uniform(1500, 3000, size=shape)
    rho = rng.uniform(0.5, 2.5, size=shape)
    return m, rho


@pytest.mark.parametrize("shape", [(9,), (6, 11), (11, 6), (4, 5, 6)])
def test_constant_density_is_a_scaled_slowness(shape):
    """rho = c everywhere: B_rho(m) = c B(m / sqrt(c)) (couplings times c,
    boundary term times sqrt(c), mass term unchanged)."""
    m, _ = _rand(shape, 2)
    h, om, al = 9.0, 2 * np.pi * 7.0, 0.04
    for c in (0.25, 1.0, 3.0):
        Br = op.operator_B(m, h, om, al, np.full(shape, c)).toarray()
        Bs = c * op.operator_B(m / np.sqrt(c), h, om, al).toarray()
        assert np.abs(Br - Bs).max() <= 1e-14 * np.abs(Bs).max()
    # rho = 1 is the constant-density operator bit for bit
    B1 = op.operator_B(m, h, om, al, np.ones(shape))
    B0 = op.operator_B(m, h, om, al)
    assert abs(B1 - B0).max() == 0.0


@pytest.mark.parametrize("shape", [(9,), (6, 11), (4, 5, 6)])
def test_density_operator_symmetric_with_neumann_null_space(shape):
    m, rho = _rand(shape, 3)
    B = op.operator_B(m, 9.0, 2 * np.pi * 7.0, 0.04, rho)
    assert abs(B - B.T).max() == 0.0
    L, g, w = op.stencil_parts(shape, rho)
    assert np.abs(L @ np.ones(L.shape[0])).max() <= 1e-15 * np.abs(L).max()
    # a coupling carries the mean density of its two nodes
    L0, _, _ = op.stencil_parts(shape)
    r = rho.ravel()
    Lc, L0c = L.tocoo(), L0.tocsr()
    off = Lc.row != Lc.col
    p, q = Lc.row[off], Lc.col[off]
    ref = np.asarray(L0c[p, q]).ravel() * 0.5 * (r[p] + r[q])
    assert np.allclose(Lc.data[off], ref, rtol=1e-15, atol=0)
    # the diagonal of L is the sum of its row's couplings, off-diagonals negative
    assert np.all(Lc.data[off] < 0)


def _rho_2d(X, Z, Lx, Lz):
    """Smooth density 1 + 0.4 sin(2 pi x / Lx) cos(pi z / Lz) and its gradient."""
    ax, az = 2 * np.pi / Lx, np.pi / Lz
    r = 1.0 + 0.4 * np.sin(ax * X) * np.cos(az * Z)
    rx = 0.4 * ax * np.cos(ax * X) * np.cos(az * Z)
    rz = -0.4 * az * np.sin(ax * X) * np.sin(az * Z)
    return r, rx, rz


def _manufactured_2d_rho(nx, nz, Lx, Lz, c, om, al):
    """u* = cos(pi x / Lx) cos(pi z / Lz) exp(-j k0 x) with a smooth density:
    f = -(rho_x u_x + rho u_xx + rho_z u_z + rho u_zz) - k^2 (1 - j alpha) u,
    and on each edge the flux condition's data rho du/dn + j omega m sqrt(rho) u."""
    h = Lx / (nx - 1)
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
    r, rx, rz = _rho_2d(X, Z, Lx, Lz)
    f = -(rx * ux + r * uxx + rz * uz + r * uzz) - k ** 2 * (1 - 1j * al) * u
    wz, wx = op.end_weights(nz), op.end_weights(nx)
    b = np.outer(wz, wx) * f
    sr = np.sqrt(r)
    b[:, 0] += wz * (-r[:, 0] * ux[:, 0] + 1j * k * sr[:, 0] * u[:, 0]) / h
    b[:, -1] += wz * (r[:, -1] * ux[:, -1] + 1j * k * sr[:, -1] * u[:, -1]) / h
    b[0, :] += wx * (-r[0, :] * uz[0, :] + 1j * k * sr[0, :] * u[0, :]) / h
    b[-1, :] += wx * (r[-1, :] * uz[-1, :] + 1j * k * sr[-1, :] * u[-1, :]) / h
    return u.ravel(), b.ravel(), r, h


def test_2d_variable_density_manufactured_second_order():
    Lx, Lz, c, f, al = 1200.0, 800.0, 2000.0, 4.0, 0.05
    om = 2 * np.pi * f
    errs = []
    for nx in (61, 121, 241):
        nz = (nx - 1) * 2 // 3 + 1
        u, b, rho, h = _manufactured_2d_rho(nx, nz, Lx, Lz, c, om, al)
        B = op.operator_B(np.full((nz, nx), 1 / c), h, om, al, rho)
        x = direct.solve_superlu(B, b)
        errs.append(np.linalg.norm(x - u) / np.linalg.norm(u))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs
    # the same data solved without the density is off by O(1): rho matters
    B1 = op.operator_B(np.full(rho.shape, 1 / c), h, om, al)
    x1 = direct.solve_superlu(B1, b)
    assert np.linalg.norm(x1 - u) / np.linalg.norm(u) > 0.05


def test_1d_variable_density_manufactured_second_order():
    """-(rho u')' - kappa^2 u = f on (0, L), rho = 2 + cos(3 pi x / L),
    u* = exp(-j k0 x) (1 + x / L), flux data at both ends."""
    Lt, c, f, al = 3000.0, 1800.0, 6.0, 0.02
    om = 2 * np.pi * f
    k = om / c
    k0 = 0.8 * k
    errs = []
    for n in (301, 601, 1201):
        h = Lt / (n - 1)
        x = np.arange(n) * h
        a = 3 * np.pi / Lt
        r, rx = 2 + np.cos(a * x), -a * np.sin(a * x)
        e = np.exp(-1j * k0 * x)
        u = e * (1 + x / Lt)
        ux = e * (-1j * k0 * (1 + x / Lt) + 1 / Lt)
        uxx = e * (-k0 ** 2 * (1 + x / Lt) - 2j * k0 / Lt)
        fx = -(rx * ux + r * uxx) - k ** 2 * (1 - 1j * al) * u
        b = op.end_weights(n) * fx
        b[0] += (-r[0] * ux[0] + 1j * k * np.sqrt(r[0]) * u[0]) / h
        b[-1] += (r[-1] * ux[-1] + 1j * k * np.sqrt(r[-1]) * u[-1]) / h
        B = op.operator_B(np.full(n, 1 / c), h, om, al, r)
        sol = direct.solve_superlu(B, b)
        errs.append(np.linalg.norm(sol - u) / np.linalg.norm(u))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, errs


def test_1d_density_jump_flux_continuity():
    """A density jump from rho1 to rho2 between two nodes: the continuum
    solution keeps u and rho u' continuous (the flux of Eq. (1)); the face mean
    converges to it (first order at a jump, so a loose bound)."""
    Lt, c, f, al = 2400.0, 2000.0, 5.0, 0.01
    rho1, rho2 = 1.0, 2.5
    om = 2 * np.pi * f
    k = om / c
    kap = k * np.sqrt(1 - 1j * al)
    xi = Lt / 2
    # in a layer of density r the wavenumber is kap / sqrt(r):
    # u = A e^{-j q x} + C e^{j q x} on each side, 4 unknowns;
    # left: -rho1 u'(0) + j k sqrt(rho1) u(0) = 1 (the unit source as a flux),
    # right: rho2 u' + j k sqrt(rho2) u = 0
    q1, q2 = kap / np.sqrt(rho1), kap / np.sqrt(rho2)
    M = np.zeros((4, 4), dtype=complex)
    rhs = np.zeros(4, dtype=complex)
    M[0] = [rho1 * 1j * q1 + 1j * k * np.sqrt(rho1), -rho1 * 1j * q1 + 1j * k * np.sqrt(rho1), 0, 0]
    rhs[0] = 1.0
    ea1, ec1 = np.exp(-1j * q1 * xi), np.exp(1j * q1 * xi)
    ea2, ec2 = np.exp(-1j * q2 * xi), np.exp(1j * q2 * xi)
    M[1] = [ea1, ec1, -ea2, -ec2]
    M[2] = [-1j * q1 * rho1 * ea1, 1j * q1 * rho1 * ec1, 1j * q2 * rho2 * ea2, -1j * q2 * rho2 * ec2]
    el, ecl = np.exp(-1j * q2 * Lt), np.exp(1j * q2 * Lt)
    M[3] = [0, 0, (-1j * q2 * rho2 + 1j * k * np.sqrt(rho2)) * el, (1j * q2 * rho2 + 1j * k * np.sqrt(rho2)) * ecl]
    co = np.linalg.solve(M, rhs)
    errs = []
    for n in (480, 960, 1920):  # even: the jump sits between two nodes
        h = Lt / (n - 1)
        x = np.arange(n) * h
        r = np.where(x < xi, rho1, rho2)
        ref = np.where(x < xi, co[0] * np.exp(-1j * q1 * x) + co[1] * np.exp(1j * q1 * x),
                       co[2] * np.exp(-1j * q2 * x) + co[3] * np.exp(1j * q2 * x))
        u = direct.solve_superlu(op.operator_B(np.full(n, 1 / c), h, om, al, r),
                                 op.point_source((n,), h, [0]))
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    assert errs[-1] < 0.01 and errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.7, errs


@pytest.mark.parametrize("shape,levels", [((17,), 3), ((9, 17), 3), ((17, 17), 3), ((10, 18), 2)])
def test_density_vcycle_equals_explicit_matrix(shape, levels):
    m, rho = _rand(shape, 5)
    vc = mg.VCycle(m, 40.0, 2 * np.pi * 6.0, 1.0, 0.5, levels, 2, 2, [0.8, 0.5][:levels - 1], rho=rho)
    C = mg.vcycle_matrix(vc)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(m.size) + 1j * rng.standard_normal(m.size)
    assert np.linalg.norm(vc(b) - C @ b) <= 1e-13 * np.linalg.norm(C @ b)
    # every level holds M of the injected slowness and density
    ml, rl, hl = m, rho, 40.0
    for l in range(levels):
        D = np.diag(op.operator_M(ml, hl, 2 * np.pi * 6.0, 1.0, 0.5, rl).toarray())
        assert np.array_equal(vc.D[l], D)
        ml, rl, hl = mg.inject(ml), mg.inject(rl), 2 * hl


@pytest.mark.parametrize("coarse", ["exact", "jacobi"])
def test_constant_density_vcycle_scales(coarse):
    """rho = c: every level's M is c M(m / sqrt(c)), Jacobi and the coarse map
    scale with it, so the cycle applied to b is the plain cycle of m / sqrt(c)
    applied to b / c."""
    shape = (17, 33)
    m, _ = _rand(shape, 6)
    c = 2.7
    kw = dict(coarse=coarse, coarse_sweeps=3, coarse_w=0.7)
    vr = mg.VCycle(m, 30.0, 2 * np.pi * 5.0, 1.0, 0.5, 3, 2, 2, [0.8, 0.6], rho=np.full(shape, c), **kw)
    v0 = mg.VCycle(m / np.sqrt(c), 30.0, 2 * np.pi * 5.0, 1.0, 0.5, 3, 2, 2, [0.8, 0.6], **kw)
    b = workloads.random_vectors(1, m.size, 4)[0]
    assert np.linalg.norm(vr(b) - v0(b / c)) <= 1e-13 * np.linalg.norm(v0(b / c))


def test_density_coarse_operator_approximates_galerkin():
    """R M_h P v ~ M_2h v for smooth v with a smooth density injected to the
    coarse level (interior, O(h^2)); without the density on the coarse level
    the gap stays O(1)."""
    errs, wrong = [], []
    for n in (33, 65, 129):
        h = 1600.0 / (n - 1)
        Z, X = np.meshgrid(np.linspace(0, 1600, n), np.linspace(0, 1600, n), indexing="ij")
        rho, _, _ = _rho_2d(X, Z, 1600.0, 1600.0)
        m = np.full((n, n), 1 / 2000.0)
        Mf = op.operator_M(m, h, 2 * np.pi * 2.0, 1.0, 0.5, rho)
        cs = mg.coarse_shape((n, n))
        Mc = op.operator_M(mg.inject(m), 2 * h, 2 * np.pi * 2.0, 1.0, 0.5, mg.inject(rho))
        M1 = op.operator_M(mg.inject(m), 2 * h, 2 * np.pi * 2.0, 1.0, 0.5)
        Zc, Xc = np.meshgrid(np.linspace(0, 1, cs[0]), np.linspace(0, 1, cs[1]), indexing="ij")
        v = (np.sin(np.pi * Xc) * np.sin(np.pi * Zc)).ravel()
        g = mg.restriction(cs) @ (Mf @ (mg.prolongation(cs) @ v))
        d = (g - Mc @ v).reshape(cs)[2:-2, 2:-2]
        ref = np.linalg.norm((Mc @ v).reshape(cs)[2:-2, 2:-2])
        errs.append(np.linalg.norm(d) / ref)
        wrong.append(np.linalg.norm((g - M1 @ v).reshape(cs)[2:-2, 2:-2]) / ref)
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert min(wrong) > 0.02 and min(wrong) > 20 * errs[-1], (wrong, errs)


def test_auto_coarse_policy_uses_density_slowness():
    """kh on the coarsest level is omega h 2^(L-1) min(m / sqrt(rho))."""
    shape = (33, 33)
    m = np.full(shape, 1 / 1500.0)
    om, h, L = 2 * np.pi * 9.0, 10.0, 4
    kh = om * h * 2 ** (L - 1) * m.min()
    assert 2.5 < kh < 2.5 * 1.3  # smoothable at rho = 1 ...
    assert mg.VCycle(m, h, om, 1.0, 0.5, L, coarse="auto").coarse == "jacobi"
    # ... not once the density lowers the wavenumber below the bound
    assert mg.VCycle(m, h, om, 1.0, 0.5, L, coarse="auto", rho=np.full(shape, 1.69)).coarse == "exact"
    assert mg.VCycle(m, h, om, 1.0, 0.5, L, coarse="auto", rho=np.full(shape, 0.5)).coarse == "jacobi"


def _density_setup(n=(21, 33), h=40.0):
    nz, nx = n
    true = workloads.model_2d_layered(nz=nz, nx=nx, h=h, nshots=3, freqs=(2.0, 3.0))
    start = workloads.model_2d_layered(nz=nz, nx=nx, h=h, nshots=3, freqs=(2.0, 3.0), seed=5)
    rho = workloads.gardner_density(true.m)
    rec = list(range(0, nx, 4)) + [nz * nx - 1]
    sv = og.Survey(true.shape, h, true.freqs, 0.05, true.src, rec, rho=rho)
    return start.m, sv, og.data(true.m, sv)


def test_density_gradient_matches_central_differences():
    m, sv, d_obs = _density_setup()
    J, g = og.gradient(m, sv, d_obs, 0.0)
    for seed in (1, 2):
        v = workloads.smooth_random_vectors(1, m.shape, seed, sigma=2.0)[0].real.reshape(m.shape)
        v = v / np.abs(v).max() * np.abs(m).max()
        eps = 1e-4
        fd = (og.misfit(m + eps * v, sv, d_obs, 0.0) - og.misfit(m - eps * v, sv, d_obs, 0.0)) / (2 * eps)
        an = float(np.sum(g * v))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    # boundary nodes: the sqrt(rho) of the absorbing term is in the gradient
    nz, nx = m.shape
    for (iz, ix) in ((0, 5), (nz - 1, 7), (4, 0), (nz - 1, nx - 1)):
        v = np.zeros_like(m)
        v[iz, ix] = m[iz, ix]
        eps = 1e-5
        fd = (og.misfit(m + eps * v, sv, d_obs, 0.0) - og.misfit(m - eps * v, sv, d_obs, 0.0)) / (2 * eps)
        assert abs(fd - g[iz, ix] * v[iz, ix]) <= 1e-5 * abs(fd) + 1e-12 * J


def test_gardner_density_range():
    w = workloads.model_2d_layered(nz=41, nx=81, h=10.0, nshots=2, freqs=(3.0,))
    rho = workloads.gardner_density(w.m)
    assert rho.shape == w.m.shape and rho.min() == 1.0 and rho.max() < 1.4


def test_3d_variable_density_manufactured_second_order():
    """Eq. (1) with d = 3: u* = cos(pi x/Lx) cos(pi y/Ly) cos(pi z/Lz)
    exp(-j k0 x) with rho = 1 + 0.3 sin(2 pi x / Lx) cos(pi y / Ly) cos(pi z / Lz),
    f = -div(rho grad u*) - k^2 (1 - j alpha) u* and on every face the flux
    data rho du*/dn + j k sqrt(rho) u*."""
    lengths, c, f, al = (600.0, 800.0, 1200.0), 2000.0, 1.5, 0.05
    Lz, Ly, Lx = lengths
    om = 2 * np.pi * f
    k = om / c
    k0 = 0.7 * k
    errs = []
    for nx in (13, 25, 49):
        shape = ((nx - 1) // 2 + 1, (nx - 1) * 2 // 3 + 1, nx)
        h = Lx / (nx - 1)
        z, y, x = (np.arange(n) * h for n in shape)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
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
        uyy = -ay ** 2 * u
        uzz = -az ** 2 * u
        a2 = 2 * np.pi / Lx
        r = 1 + 0.3 * np.sin(a2 * X) * cy * cz
        rx = 0.3 * a2 * np.cos(a2 * X) * cy * cz
        ry = -0.3 * ay * np.sin(a2 * X) * sy * cz
        rz = -0.3 * az * np.sin(a2 * X) * cy * sz
        fs = -(rx * ux + ry * uy + rz * uz + r * (uxx + uyy + uzz)) - k ** 2 * (1 - 1j * al) * u
        wz, wy, wx = (op.end_weights(n) for n in shape)
        b = wz[:, None, None] * wy[None, :, None] * wx[None, None, :] * fs
        fx = wz[:, None] * wy[None, :]
        fy = wz[:, None] * wx[None, :]
        fz = wy[:, None] * wx[None, :]
        sr = np.sqrt(r)
        b[:, :, 0] += fx * (-r[:, :, 0] * ux[:, :, 0] + 1j * k * sr[:, :, 0] * u[:, :, 0]) / h
        b[:, :, -1] += fx * (r[:, :, -1] * ux[:, :, -1] + 1j * k * sr[:, :, -1] * u[:, :, -1]) / h
        b[:, 0, :] += fy * (-r[:, 0, :] * uy[:, 0, :] + 1j * k * sr[:, 0, :] * u[:, 0, :]) / h
        b[:, -1, :] += fy * (r[:, -1, :] * uy[:, -1, :] + 1j * k * sr[:, -1, :] * u[:, -1, :]) / h
        b[0, :, :] += fz * (-r[0, :, :] * uz[0, :, :] + 1j * k * sr[0, :, :] * u[0, :, :]) / h
        b[-1, :, :] += fz * (r[-1, :, :] * uz[-1, :, :] + 1j * k * sr[-1, :, :] * u[-1, :, :]) / h
        B = op.operator_B(np.full(shape, 1 / c), h, om, al, r)
        sol = direct.solve_superlu(B, b.ravel())
        errs.append(np.linalg.norm(sol - u.ravel()) / np.linalg.norm(u))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.6 < r2 < 4.4, errs


def test_3d_density_vcycle_equals_explicit_matrix():
    shape = (9, 9, 17)
    m, rho = _rand(shape, 12)
    vc = mg.VCycle(m, 40.0, 2 * np.pi * 4.0, 1.0, 0.5, 2, 2, 2, [0.7], rho=rho)
    C = mg.vcycle_matrix(vc)
    b = workloads.random_vectors(1, m.size, 13)[0]
    assert np.linalg.norm(vc(b) - C @ b) <= 1e-13 * np.linalg.norm(C @ b)
    D = np.diag(op.operator_M(mg.inject(m), 80.0, 2 * np.pi * 4.0, 1.0, 0.5, mg.inject(rho)).toarray())
    assert np.array_equal(vc.D[1], D)


def test_3d_density_gradient_matches_central_differences():
    nz, ny, nx, h = 7, 9, 11, 50.0
    true = workloads.model_3d_layered(nz=nz, ny=ny, nx=nx, h=h, nshots=2, freqs=(2.0,))
    start = workloads.model_3d_layered(nz=nz, ny=ny, nx=nx, h=h, nshots=2, freqs=(2.0,), seed=4)
    rho = workloads.gardner_density(true.m)
    src = [(s[0] * ny + s[1]) * nx + s[2] for s in true.src]
    rec = list(range(0, ny * nx, 5)) + [nz * ny * nx - 1]
    sv = og.Survey(true.shape, h, true.freqs, 0.05, src, rec, rho=rho)
    d_obs = og.data(true.m, sv)
    m = start.m
    J, g = og.gradient(m, sv, d_obs, 0.0)
    for (iz, iy, ix) in ((0, 4, 5), (3, 4, 5), (nz - 1, 0, nx - 1)):
        v = np.zeros_like(m)
        v[iz, iy, ix] = m[iz, iy, ix]
        eps = 1e-5
        fd = (og.misfit(m + eps * v, sv, d_obs, 0.0) - og.misfit(m - eps * v, sv, d_obs, 0.0)) / (2 * eps)
        assert abs(fd - g[iz, iy, ix] * v[iz, iy, ix]) <= 1e-5 * abs(fd) + 1e-12 * J
