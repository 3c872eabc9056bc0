"""Pins of the oracle's V-cycle and its level/weight plan: exactness of the
transfer operators on the functions they must reproduce, the explicit
error-propagation matrix of the cycle, the one-level case, and local Fourier
analysis checked by brute force and against the smoother's measured growth."""

import numpy as np
import pytest

from oracle import operator as op
from oracle import multigrid as mg
from oracle import lfa
from oracle import direct


def test_prolongation_reproduces_bilinear_functions():
    for coarse in [(5,), (5, 9), (9, 5)]:
        P = mg.prolongation(coarse)
        fine = tuple(2 * (n - 1) + 1 for n in coarse)
        if len(coarse) == 1:
            xc = np.arange(coarse[0]) * 2.0
            xf = np.arange(fine[0]) * 1.0
            fc, ff = 3 + 0.5 * xc, 3 + 0.5 * xf
        else:
            Zc, Xc = np.meshgrid(np.arange(coarse[0]) * 2.0, np.arange(coarse[1]) * 2.0, indexing="ij")
            Zf, Xf = np.meshgrid(np.arange(fine[0]) * 1.0, np.arange(fine[1]) * 1.0, indexing="ij")
            fc = 1 + 0.3 * Xc - 0.7 * Zc + 0.1 * Xc * Zc
            ff = 1 + 0.3 * Xf - 0.7 * Zf + 0.1 * Xf * Zf
        assert np.allclose(P @ fc.ravel(), ff.ravel(), rtol=0, atol=1e-12)


def test_prolongation_on_even_count_axes():
    """An axis with an even node count: linear functions are reproduced at
    every fine node but the last, which takes the last coarse value."""
    for coarse, fine in [((5,), (10,)), ((5, 9), (10, 17)), ((5, 9), (9, 18)), ((4, 4), (8, 7))]:
        P = mg.prolongation(coarse, fine)
        Zc, Xc = np.meshgrid(np.arange(coarse[0]) * 2.0, np.arange(coarse[-1]) * 2.0, indexing="ij")
        Zf, Xf = np.meshgrid(np.arange(fine[0]) * 1.0, np.arange(fine[-1]) * 1.0, indexing="ij")
        if len(coarse) == 1:
            Zc, Zf = np.zeros_like(Xc[:1]), np.zeros_like(Xf[:1])
            Xc, Xf = Xc[:1], Xf[:1]
        fc = 1 + 0.3 * Xc - 0.7 * Zc + 0.1 * Xc * Zc
        ff = 1 + 0.3 * Xf - 0.7 * Zf + 0.1 * Xf * Zf
        # the fine coordinate of the extra node moves onto the last coarse node
        Xe = np.minimum(Xf, 2.0 * (coarse[-1] - 1))
        Ze = np.minimum(Zf, 2.0 * (coarse[0] - 1)) if len(coarse) == 2 else Zf
        fe = 1 + 0.3 * Xe - 0.7 * Ze + 0.1 * Xe * Ze
        got = (P @ fc.ravel()).reshape(ff.shape)
        assert np.allclose(got, fe, rtol=0, atol=1e-12)
        inner = (Xf <= 2.0 * (coarse[-1] - 1)) & (Zf <= 2.0 * (coarse[0] - 1))
        assert np.allclose(got[inner], ff[inner], rtol=0, atol=1e-12)


def test_restriction_weighted_constants_on_even_count_axes():
    """With an even node count the last coarse node collects the whole last
    fine cell: R (W_fine 1) equals the coarse weights except on that node,
    where the axis weight is 1 instead of 1/2."""
    for coarse, fine in [((5,), (10,)), ((5, 9), (10, 17)), ((5, 9), (9, 18))]:
        _, _, wf = op.stencil_parts(fine)
        _, _, wc = op.stencil_parts(coarse)
        got = (mg.restriction(coarse, fine) @ wf).reshape(coarse)
        exp = wc.reshape(coarse).copy()
        axes = [(a, n) for a, (n, nf) in enumerate(zip(coarse, fine)) if nf % 2 == 0]
        for a, n in axes:
            idx = [slice(None)] * len(coarse)
            idx[a] = n - 1
            exp[tuple(idx)] *= 2.0
        assert np.allclose(got, exp, rtol=0, atol=1e-14)


def test_restriction_preserves_weighted_constants():
    """R (W_fine 1) = W_coarse 1: the weighted residual keeps its meaning."""
    for coarse in [(5,), (5, 9), (9, 5), (3, 3)]:
        fine = tuple(2 * (n - 1) + 1 for n in coarse)
        _, _, wf = op.stencil_parts(fine)
        _, _, wc = op.stencil_parts(coarse)
        R = mg.restriction(coarse)
        assert np.allclose(R @ wf, wc, rtol=0, atol=1e-14)


def test_full_weighting_in_the_interior():
    R = mg.restriction((5, 5)).toarray()
    row = R[2 * 5 + 2].reshape(9, 9)
    ref = np.zeros((9, 9))
    ref[3:6, 3:6] = np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]) / 16.0
    assert np.array_equal(row, ref)


def test_coarse_operator_approximates_galerkin_on_smooth_vectors():
    """R M_h P v ~ M_2h v for smooth v (interior, O(h^2))."""
    errs = []
    for n in (33, 65, 129):
        h = 1600.0 / (n - 1)
        m = np.full((n, n), 1 / 2000.0)
        Mf = op.operator_M(m, h, 2 * np.pi * 2.0, 1.0, 0.5)
        cs = mg.coarse_shape((n, n))
        Mc = op.operator_M(mg.inject(m), 2 * h, 2 * np.pi * 2.0, 1.0, 0.5)
        Z, X = np.meshgrid(np.linspace(0, 1, cs[0]), np.linspace(0, 1, cs[1]), indexing="ij")
        v = (np.sin(np.pi * X) * np.sin(np.pi * Z)).ravel()
        g = mg.restriction(cs) @ (Mf @ (mg.prolongation(cs) @ v))
        d = (g - Mc @ v).reshape(cs)[2:-2, 2:-2]
        errs.append(np.linalg.norm(d) / np.linalg.norm((Mc @ v).reshape(cs)[2:-2, 2:-2]))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


@pytest.mark.parametrize("shape,levels,nu", [((16,), 3, (2, 2)), ((10, 18), 3, (1, 1)),
                                             ((17,), 3, (2, 2)), ((17, 17), 3, (2, 2)),
                                            ((9, 17), 3, (1, 1)), ((17, 9), 2, (2, 1))])
def test_vcycle_equals_explicit_error_propagation(shape, levels, nu):
    rng = np.random.default_rng(5)
    m = 1 / rng.uniform(1500, 3000, size=shape)
    h, om = 40.0, 2 * np.pi * 6.0
    wj = [0.8, 0.5, 0.3][:levels - 1]
    vc = mg.VCycle(m, h, om, 1.0, 0.5, levels, nu[0], nu[1], wj)
    C = mg.vcycle_matrix(vc)
    b = rng.standard_normal(C.shape[0]) + 1j * rng.standard_normal(C.shape[0])
    assert np.linalg.norm(vc(b) - C @ b) <= 1e-13 * np.linalg.norm(C @ b)
    # the V-cycle is linear and its matrix is not the exact inverse
    Minv = np.linalg.inv(vc.M[0].toarray())
    assert np.linalg.norm(C - Minv) > 1e-6 * np.linalg.norm(Minv)


@pytest.mark.parametrize("shape", [(17, 17), (10, 18)])
def test_vcycle_with_jacobi_coarse_level(shape):
    """Coarsest level smoothed (k sweeps from zero) instead of solved: the
    cycle equals the error-propagation matrix with (I - S^k) M_c^-1 there."""
    rng = np.random.default_rng(8)
    m = 1.0 / rng.uniform(1500, 3000, size=shape)
    vc = mg.VCycle(m, 40.0, 2 * np.pi * 6.0, 1.0, 0.5, 3, 2, 2, [0.8, 0.7], coarse="jacobi", coarse_sweeps=5)
    C = mg.vcycle_matrix(vc)
    b = rng.standard_normal(m.size) + 1j * rng.standard_normal(m.size)
    assert np.allclose(vc(b), C @ b, rtol=1e-11, atol=1e-14 * np.abs(C @ b).max())


def test_jacobi_converges_on_coarse_level_at_large_kh():
    """Damped Jacobi (w = 0.8) on the shifted Laplacian (1, 0.5) contracts
    every mode when the level's smallest kh is >= 2.5 (brute-force spectral
    radius of the iteration matrix), but not at small kh."""
    for n, h, f, contracts in [(9, 320.0, 12.0, True), (9, 320.0, 8.0, True), (9, 320.0, 1.0, False)]:
        m = np.full((n, n), 1 / 3000.0)
        kh_min = 2 * np.pi * f * h * m.min()
        M = op.operator_M(m, h, 2 * np.pi * f, 1.0, 0.5).toarray()
        S = np.eye(n * n) - 0.8 * M / np.diag(M)[:, None]
        rho = np.abs(np.linalg.eigvals(S)).max()
        assert (kh_min >= 2.5) == contracts
        assert (rho < 1.0) == contracts, (f, kh_min, rho)


def test_one_level_is_exact_inverse_of_M():
    rng = np.random.default_rng(6)
    m = 1 / rng.uniform(1500, 3000, size=(201,))
    vc = mg.VCycle(m, 5.0, 2 * np.pi * 10.0, 1.0, 0.5, 1)
    b = rng.standard_normal(201) + 1j * rng.standard_normal(201)
    x = vc(b)
    M = op.operator_M(m, 5.0, 2 * np.pi * 10.0, 1.0, 0.5)
    assert np.linalg.norm(M @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - direct.solve_dense(M, b)) <= 1e-12 * np.linalg.norm(x)


def test_vcycle_solves_low_frequency_problem_as_iteration():
    """At low kh the V-cycle contracts the error of M u = b strongly."""
    n = 65
    m = np.full((n, n), 1 / 2000.0)
    h, om = 10.0, 2 * np.pi * 3.0
    vc = mg.VCycle(m, h, om, 1.0, 0.5, 4, 2, 2, [0.8] * 3)
    M = vc.M[0]
    rng = np.random.default_rng(2)
    b = rng.standard_normal(n * n) + 0j
    u = np.zeros_like(b)
    res = []
    for _ in range(6):
        u = u + vc(b - M @ u)
        res.append(np.linalg.norm(b - M @ u))
    assert res[-1] / res[0] < 1e-4


def test_lfa_closed_form_matches_brute_force():
    for kh in (0.1, 0.6, 1.2, 1.84, 2.3, 3.5):
        for (b1, b2, w) in ((1, 0.5, 0.8), (1, 1, 0.8), (1, 0.5, 0.4)):
            a = lfa.smoothing_factor(kh, b1, b2, w, 2)
            bf = lfa.smoothing_factor_sampled(kh, b1, b2, w, 2, n=257)
            assert abs(a - bf) < 1e-12
            a1 = lfa.smoothing_factor(kh, b1, b2, w, 1)
            bf1 = lfa.smoothing_factor_sampled(kh, b1, b2, w, 1, n=2049)
            assert abs(a1 - bf1) < 1e-12


def test_lfa_bad_band_for_half_shift():
    """Damped Jacobi w = 0.8 on the (1, 0.5) shifted Laplacian amplifies
    high-frequency errors for kh between about 1.19 and 2.46."""
    khs = np.linspace(0.01, 5, 4991)
    mu = np.array([lfa.smoothing_factor(k, 1, 0.5, 0.8) for k in khs])
    bad = khs[mu > 1]
    assert abs(bad.min() - 1.19) < 0.01 and abs(bad.max() - 2.46) < 0.01
    assert abs(mu.max() - 1.719) < 1e-3
    assert max(lfa.smoothing_factor(k, 1, 0.5, 0.3) for k in khs) < 1


@pytest.mark.parametrize("kh,grows", [(0.4, False), (1.84, True), (3.5, False)])
def test_smoother_growth_matches_lfa(kh, grows):
    """Jacobi sweeps on M u = 0 from a checkerboard error: the per-sweep growth
    of the interior error follows the LFA factor at theta = (pi, pi)."""
    n, h = 129, 10.0
    c = 2000.0
    om = kh * c / h
    m = np.full((n, n), 1 / c)
    M = op.operator_M(m, h, om, 1.0, 0.5)
    D = M.diagonal()
    iz, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = ((-1.0) ** (iz + ix)).ravel().astype(complex)
    inner = ((iz > 20) & (iz < n - 21) & (ix > 20) & (ix < n - 21)).ravel()
    norms = []
    for _ in range(8):
        u = u - 0.8 * (M @ u) / D
        norms.append(np.linalg.norm(u[inner]))
    rate = norms[-1] / norms[-2]
    s = complex(1, -0.5)
    q = kh ** 2
    pred = abs(1 - 0.8 * (8 - s * q) / (4 - s * q))
    assert abs(rate - pred) < 1e-6
    assert (rate > 1) == grows


def test_plan_levels_and_weights():
    # default plans: halve while the coarsest level has more than 512 unknowns
    assert lfa.default_levels((201, 201)) == 5   # ... 26 x 26 -> 13 x 13
    assert lfa.default_levels((401, 801)) == 6   # ... 26 x 51 -> 13 x 26
    assert lfa.default_levels((301, 601)) == 6   # 76 x 151 -> 38 x 76 -> 19 x 38 -> 10 x 19
    assert lfa.default_levels((129, 129)) == 4   # 17 x 17
    assert lfa.default_levels((1001,)) == 2
    assert lfa.default_levels((17, 17)) == 1
    assert lfa.max_levels((301, 601)) == 8       # ... 10 x 19 -> 5 x 10 -> 3 x 5
    assert lfa.max_levels((1001,)) == 9
    assert mg.coarse_shape((76, 151)) == (38, 76)
    # low kh everywhere: the default weight is kept
    L, w = lfa.plan((201, 201), 10.0, 2 * np.pi * 5, 1 / 2800, 1 / 1200, 1, 0.5, levels=4)
    assert L == 4 and w == [0.8, 0.8, 0.8]
    # a level in the band gets a smaller weight with mu <= 1 over its kh range
    L, w = lfa.plan((401, 801), 10.0, 2 * np.pi * 12, 1 / 5175, 1 / 1275, 1, 0.5)
    assert L == 6 and w[0] == 0.8 and w[2] < 0.8
    for l, wl in enumerate(w):
        hl = 10.0 * 2 ** l
        for kh in np.linspace(2 * np.pi * 12 * hl / 5175, 2 * np.pi * 12 * hl / 1275, 200):
            assert lfa.smoothing_factor(kh, 1, 0.5, wl) <= 1.0 + 1e-3
