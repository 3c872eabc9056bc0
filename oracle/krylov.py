"""ORACLE (test infrastructure only): right-preconditioned Krylov solvers.

The paper models its data with a Krylov subspace method (GMRES) preconditioned
by the shifted-Laplace operator (section on FWI; Examples; Conclusion). The
solvers here are the textbook ones, with x0 = 0, the Hermitian inner product
<a, b> = sum conj(a_i) b_i, and the stopping test ||r||_2 <= tol ||b||_2:

* BiCGSTAB (van der Vorst, 1992), preconditioned on the right: the residual it
  updates is the true residual b - A x. The test is made after each full
  step. On a breakdown (rho, <rhat, v> or omega exactly zero) the method is
  restarted once from the current iterate with the shadow vector rhat = r;
  a second breakdown, or any non-finite scalar, stops it.
* GMRES(m) (Saad and Schultz, 1986), preconditioned on the right, modified
  Gram-Schmidt Arnoldi with complex Givens rotations, tested on the Arnoldi
  residual estimate at every inner step; each cycle ends with
  x += M^-1 (V y) and the true residual.

Both count one iteration per pass of the loop (BiCGSTAB: two preconditioner
applications and two operator applications; GMRES: one of each) and report
the true relative residual ||b - A x|| / ||b|| of the returned x.
"""

import numpy as np

CONVERGED, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3


def _as_op(A):
    return A if callable(A) else (lambda x: A @ x)


def bicgstab(A, b, M=None, tol=1e-8, maxit=1000, rhat=None, history=None):
    """Return (x, iterations, true relative residual, status)."""
    Aop = _as_op(A)
    Mop = M if M is not None else (lambda x: x)
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0:
        return x, 0, 0.0, CONVERGED
    r = b.copy()
    rh = b.copy() if rhat is None else np.asarray(rhat, dtype=np.complex128).copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    restarted = False
    it = 0
    status = MAXIT

    def restart():
        nonlocal rh, rho, alpha, omega, v, p, restarted
        rh = r.copy()
        rho = alpha = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        restarted = True

    while it < maxit:
        rho_new = np.vdot(rh, r)
        if not np.isfinite(rho_new):
            status = NONFINITE
            break
        if rho_new == 0:
            if restarted:
                status = BREAKDOWN
                break
            restart()
            continue
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        ph = Mop(p)
        v = Aop(ph)
        sigma = np.vdot(rh, v)
        if not np.isfinite(sigma):
            status = NONFINITE
            break
        if sigma == 0:
            if restarted:
                status = BREAKDOWN
                break
            restart()
            continue
        alpha = rho / sigma
        s = r - alpha * v
        sh = Mop(s)
        t = Aop(sh)
        tt = np.vdot(t, t)
        omega = np.vdot(t, s) / tt if tt != 0 else 0.0 + 0j
        if not (np.isfinite(alpha) and np.isfinite(omega)):
            status = NONFINITE
            break
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        it += 1
        rn = np.linalg.norm(r)
        if history is not None:
            history.append(rn / bnorm)
        if not np.isfinite(rn):
            status = NONFINITE
            break
        if rn <= tol * bnorm:
            status = CONVERGED
            break
        if omega == 0:
            if restarted:
                status = BREAKDOWN
                break
            restart()
    relres = np.linalg.norm(b - Aop(x)) / bnorm
    return x, it, relres, status


def _givens(a, b):
    """Complex rotation (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0j
    if a == 0:
        return 0.0, 1.0 + 0j
    nu = np.hypot(abs(a), abs(b))
    c = abs(a) / nu
    s = (a / abs(a)) * np.conj(b) / nu
    return c, s


def gmres(A, b, M=None, m=30, tol=1e-8, maxit=1000, history=None):
    """Return (x, iterations, true relative residual, status)."""
    Aop = _as_op(A)
    Mop = M if M is not None else (lambda x: x)
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0:
        return x, 0, 0.0, CONVERGED
    r = b.copy()
    beta = bnorm
    it = 0
    status = MAXIT
    while it < maxit:
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        k = 0
        done = False
        for j in range(m):
            w = Aop(Mop(V[j]))
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * c
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            if history is not None:
                history.append(abs(g[j + 1]) / bnorm)
            if not np.isfinite(g[j + 1]):
                status = NONFINITE
                done = True
                break
            if abs(g[j + 1]) <= tol * bnorm or it >= maxit:
                break
        if status == NONFINITE:
            break
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + Mop(V[:k].T @ y)
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            status = CONVERGED
            break
        if done:
            break
    relres = np.linalg.norm(b - Aop(x)) / bnorm
    return x, it, relres, status
