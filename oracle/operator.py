"""ORACLE (test infrastructure only): the discrete Helmholtz operator.

Paper, section "Full waveform inversion in the space-frequency domain":
Eq. (2) is the constant-density Helmholtz equation
    -Laplace(u) - omega^2 m^2 (1 - j alpha) u = f,
with m = 1/c the real slowness and alpha the damping; Eq. (1) states that the
equation carries a first-order absorbing boundary condition; Eq. (3) writes
the discretised problem as B u = f.

Readings of what the paper leaves open (each listed in the design doc):

* Grid: nodes (iz, ix) at z = iz h, x = ix h, flat index iz*nx + ix; every
  edge of the rectangle absorbs. In 1D the single axis is x.
* Absorbing condition: du/dn + j omega m u = 0 on the boundary (n the outward
  normal, undamped wavenumber). Second-order centred differences; the ghost
  node beyond an edge is eliminated with the centred form of the condition.
* Each row is then multiplied by its control-volume weight w = w_x w_z, with
  w_axis = 1/2 on the two end nodes of an axis and 1 elsewhere. The result is
  the complex-symmetric matrix
      A = L / h^2 + (j omega / h) diag(g m) - omega^2 s diag(w m^2),
  where L is the real symmetric Neumann Laplacian whose coupling between two
  neighbours along one axis is the weight of the other axis, and g sums, over
  the axes on which a node is an end node, the weight of the other axis.
  s = 1 - j alpha gives B; s = beta1 - j beta2 gives the shifted Laplacian M
  (same boundary term).
* A unit point source at node p is b = e_p / h^dim in this weighted system.
"""

import numpy as np
import scipy.sparse as sp


def end_weights(n):
    """Control-volume weight along one axis: 1/2 at both end nodes, else 1."""
    w = np.ones(n)
    w[0] = 0.5
    w[-1] = 0.5
    return w


def stencil_parts(shape):
    """Return (L, g, w) for a grid of the given shape (n,) or (nz, nx).

    L is the weighted Neumann Laplacian without the 1/h^2 factor (sparse,
    real, symmetric), g the boundary-term weight and w the mass weight, both
    flattened in the grid's flat order.
    """
    if len(shape) == 1:
        (n,) = shape
        p = np.arange(n - 1)
        q = p + 1
        c = np.ones(n - 1)
        g = np.zeros(n)
        g[0] = 1.0
        g[-1] = 1.0
        w = end_weights(n)
        size = n
    else:
        nz, nx = shape
        wz, wx = end_weights(nz), end_weights(nx)
        idx = np.arange(nz * nx).reshape(nz, nx)
        # neighbours along x share the row's z-weight
        px, qx = idx[:, :-1].ravel(), idx[:, 1:].ravel()
        cx = np.repeat(wz, nx - 1)
        # neighbours along z share the column's x-weight
        pz, qz = idx[:-1, :].ravel(), idx[1:, :].ravel()
        cz = np.tile(wx, nz - 1)
        p = np.concatenate([px, pz])
        q = np.concatenate([qx, qz])
        c = np.concatenate([cx, cz])
        g2 = np.zeros((nz, nx))
        g2[:, 0] += wz
        g2[:, -1] += wz
        g2[0, :] += wx
        g2[-1, :] += wx
        g = g2.ravel()
        w = np.outer(wz, wx).ravel()
        size = nz * nx
    off = sp.coo_matrix((np.concatenate([-c, -c]),
                         (np.concatenate([p, q]), np.concatenate([q, p]))),
                        shape=(size, size))
    deg = np.bincount(p, weights=c, minlength=size) + \
        np.bincount(q, weights=c, minlength=size)
    L = (off + sp.diags(deg)).tocsr()
    return L, g, w


def helmholtz_matrix(m, h, omega, s):
    """A = L/h^2 + (j omega/h) diag(g m) - omega^2 s diag(w m^2), CSR complex128.

    m: slowness, shape (n,) for 1D or (nz, nx) for 2D. s: complex mass shift;
    s = 1 - j alpha is the operator B of Eq. (2)-(3), s = beta1 - j beta2 the
    shifted Laplacian M.
    """
    m = np.asarray(m, dtype=np.float64)
    L, g, w = stencil_parts(m.shape)
    mf = m.ravel()
    diag = 1j * omega * g * mf / h - omega ** 2 * complex(s) * w * mf ** 2
    return (L.astype(np.complex128) / h ** 2 + sp.diags(diag)).tocsr()


def operator_B(m, h, omega, alpha):
    """The damped Helmholtz operator B of Eq. (2)-(3)."""
    return helmholtz_matrix(m, h, omega, 1.0 - 1j * alpha)


def operator_M(m, h, omega, beta1, beta2):
    """The shifted-Laplace operator M = -Laplace - (beta1 - j beta2) omega^2 m^2."""
    return helmholtz_matrix(m, h, omega, beta1 - 1j * beta2)


def point_source(shape, h, nodes, amps=None):
    """Weighted right-hand side of unit (or amp-scaled) point sources.

    nodes: list of flat indices; returns a complex128 vector with amp/h^dim at
    each node (values add if a node repeats).
    """
    size = int(np.prod(shape))
    b = np.zeros(size, dtype=np.complex128)
    if amps is None:
        amps = np.ones(len(nodes), dtype=np.complex128)
    for p, a in zip(nodes, amps):
        b[int(p)] += complex(a) / h ** len(shape)
    return b
