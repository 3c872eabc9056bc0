"""Pins of the oracle's Krylov solvers: iterate-by-iterate agreement with
SciPy's BiCGSTAB (the same right-preconditioned recurrence) and GMRES (on the
right-preconditioned operator), convergence to the direct solution, the
preconditioner's effect, and the failure paths."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operator as op
from oracle import multigrid as mg
from oracle import krylov
from oracle import direct
import workloads


def _small_problem(n=65, f=5.0, sign=-1.0):
    w = workloads.model_2d_lens(n=n, h=10.0 * 200 / (n - 1), sign=sign)
    om = 2 * np.pi * f
    B = op.operator_B(w.m, w.h, om, w.alpha)
    b = op.point_source(w.shape, w.h, w.src)
    V = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 3, 2, 2, [0.8, 0.8])
    return B, b, V


def test_bicgstab_iterates_match_scipy():
    B, b, V = _small_problem()
    Mop = spla.LinearOperator(B.shape, matvec=V, dtype=np.complex128)
    for k in (1, 3, 6):
        xs, _ = spla.bicgstab(B, b, rtol=1e-30, atol=0.0, maxiter=k, M=Mop)
        xo, it, _, st = krylov.bicgstab(B, b, V, tol=1e-30, maxit=k)
        assert it == k and st == krylov.MAXIT
        assert np.linalg.norm(xo - xs) <= 1e-10 * np.linalg.norm(xs)


def test_gmres_cycle_matches_scipy_on_right_preconditioned_operator():
    B, b, V = _small_problem()
    BV = spla.LinearOperator(B.shape, matvec=lambda y: B @ V(y), dtype=np.complex128)
    m = 8
    ys, _ = spla.gmres(BV, b, rtol=1e-30, atol=0.0, restart=m, maxiter=1)
    xo, it, _, _ = krylov.gmres(B, b, V, m=m, tol=1e-30, maxit=m)
    assert it == m
    assert np.linalg.norm(xo - V(ys)) <= 1e-9 * np.linalg.norm(xo)
    # unpreconditioned, two restart cycles
    xs, _ = spla.gmres(B, b, rtol=1e-30, atol=0.0, restart=m, maxiter=2)
    xo, it, _, _ = krylov.gmres(B, b, None, m=m, tol=1e-30, maxit=2 * m)
    assert np.linalg.norm(xo - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("solver", ["bicgstab", "gmres"])
def test_converges_to_direct_solution(solver):
    B, b, V = _small_problem()
    u = direct.solve_superlu(B, b)
    fn = krylov.bicgstab if solver == "bicgstab" else krylov.gmres
    x, it, rr, st = fn(B, b, V, tol=1e-11, maxit=400)
    assert st == krylov.CONVERGED and rr <= 1e-11
    assert np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)


def test_gmres_residual_estimate_non_increasing():
    B, b, V = _small_problem()
    hist = []
    krylov.gmres(B, b, V, m=10, tol=1e-10, maxit=200, history=hist)
    # within each restart cycle the Arnoldi residual estimate cannot grow
    for j in range(0, len(hist) - 1):
        if (j + 1) % 10:
            assert hist[j + 1] <= hist[j] * (1 + 1e-12)


def test_preconditioner_accelerates_convergence():
    """The shifted-Laplace V-cycle turns a non-converging solve into a fast one
    (the paper reports a much faster convergence with the preconditioner)."""
    w = workloads.model_2d_lens()
    om = 2 * np.pi * w.freqs[0]
    B = op.operator_B(w.m, w.h, om, w.alpha)
    b = op.point_source(w.shape, w.h, w.src)
    V = mg.VCycle(w.m, w.h, om, 1.0, 0.5, 4, 2, 2, [0.8] * 3)
    _, it_p, rr_p, st_p = krylov.bicgstab(B, b, V, tol=1e-8, maxit=200)
    _, it_n, rr_n, st_n = krylov.bicgstab(B, b, None, tol=1e-8, maxit=1500)
    assert st_p == krylov.CONVERGED and it_p < 40
    assert st_n != krylov.CONVERGED and rr_n > 1e-6


def test_breakdown_restart_with_orthogonal_shadow_vector():
    """A shadow vector exactly orthogonal to b (zero where the point source is)
    makes rho zero at once; the restart with rhat = r then runs exactly the
    default iteration."""
    B, b, V = _small_problem()
    rng = np.random.default_rng(0)
    z = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    z[b != 0] = 0
    assert np.vdot(z, b) == 0
    x0, it0, _, st0 = krylov.bicgstab(B, b, V, tol=1e-10, maxit=100)
    x1, it1, _, st1 = krylov.bicgstab(B, b, V, tol=1e-10, maxit=100, rhat=z)
    assert st0 == st1 == krylov.CONVERGED and it0 == it1
    assert np.array_equal(x0, x1)
    # an operator with zero image makes <rhat, v> vanish before and after the
    # restart: the second breakdown stops the solver
    _, it, _, st = krylov.bicgstab(lambda v: 0 * v, b, None, tol=1e-10, maxit=10)
    assert st == krylov.BREAKDOWN and it == 0


def test_failure_paths():
    B, b, V = _small_problem()
    x, it, rr, st = krylov.bicgstab(B, np.zeros_like(b), V)
    assert it == 0 and st == krylov.CONVERGED and not np.any(x)
    x, it, rr, st = krylov.bicgstab(B, b, V, tol=1e-12, maxit=1)
    assert it == 1 and st == krylov.MAXIT
    bn = b.copy()
    bn[5] = np.nan
    _, _, _, st = krylov.bicgstab(B, bn, V)
    assert st == krylov.NONFINITE
    x, it, rr, st = krylov.gmres(B, np.zeros_like(b), V)
    assert it == 0 and st == krylov.CONVERGED
