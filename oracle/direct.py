"""ORACLE (test infrastructure only): direct solves of B u = f.

The paper generates its observed data by an LU factorisation of the
finite-difference system (Examples section, both the 1D well example and the
2D surface example). The oracle's reference solution of every linear system is
therefore the plain direct solve:

* ``solve_superlu``: SciPy's SuperLU (a library primitive used as one step);
* ``solve_banded``: an own banded LU with partial pivoting, the shorter grid
  axis ordered fastest so the half-bandwidth is min(nz, nx);
* ``solve_dense``: numpy.linalg.solve for tiny grids.

The three are cross-checked on small grids in the tests.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve_superlu(A, b):
    """x = A^-1 b by SuperLU; b may be (n,) or (n, k)."""
    lu = spla.splu(sp.csc_matrix(A))
    return lu.solve(np.asarray(b, dtype=np.complex128))


def factor_superlu(A):
    """SuperLU factor object (reuse for many right-hand sides)."""
    return spla.splu(sp.csc_matrix(A))


def solve_dense(A, b):
    """x = A^-1 b with numpy's dense LAPACK solve (tiny systems only)."""
    return np.linalg.solve(A.toarray(), np.asarray(b, dtype=np.complex128))


def _transpose_perm(nz, nx):
    """Permutation that orders a (nz, nx) grid with z fastest."""
    return np.arange(nz * nx).reshape(nz, nx).T.ravel()


def solve_banded(A, b, shape):
    """Own banded LU with partial pivoting (row interchanges).

    The nodes are reordered so the shorter axis is fastest; the matrix then
    has lower and upper half-bandwidth kl = ku = min(nz, nx) (1 in 1D). Row
    interchanges let the upper factor grow to bandwidth kl + ku, so row i is
    kept as a window R[i, j - i + kl] over columns j in [i - kl, i + kl + ku].
    Step k eliminates column k from rows k+1..k+kl after choosing the pivot
    of largest modulus among rows k..k+kl. Intended for small grids: the
    Python loop runs once per unknown.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    if len(shape) == 2:
        kl = min(shape)
        perm = _transpose_perm(*shape) if shape[0] < shape[1] else np.arange(n)
    else:
        kl = 1
        perm = np.arange(n)
    ku = kl
    width = 2 * kl + ku + 1
    Ap = A[perm][:, perm].tocoo()
    if np.any(np.abs(Ap.col - Ap.row) > kl):
        raise ValueError("banded LU: matrix wider than the grid band")
    R = np.zeros((n, width), dtype=np.complex128)
    R[Ap.row, Ap.col - Ap.row + kl] = Ap.data
    rhs = np.array(np.asarray(b, dtype=np.complex128)[perm], copy=True)
    for k in range(n):
        rows = np.arange(k, min(n - 1, k + kl) + 1)
        cols = np.arange(k, min(n - 1, k + kl + ku) + 1)
        off = cols[None, :] - rows[:, None] + kl
        blk = R[rows[:, None], off]
        p = int(np.argmax(np.abs(blk[:, 0])))
        if blk[p, 0] == 0:
            raise np.linalg.LinAlgError("banded LU: singular matrix")
        if p != 0:
            blk[[0, p]] = blk[[p, 0]]
            rhs[[k, k + p]] = rhs[[k + p, k]]
        f = blk[1:, 0] / blk[0, 0]
        blk[1:] -= f[:, None] * blk[0][None, :]
        rhs[rows[1:]] -= f * rhs[k]
        R[rows[:, None], off] = blk
    x = np.zeros(n, dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        cols = np.arange(i + 1, min(n - 1, i + kl + ku) + 1)
        x[i] = (rhs[i] - np.dot(R[i, cols - i + kl], x[cols])) / R[i, kl]
    out = np.empty(n, dtype=np.complex128)
    out[perm] = x
    return out
