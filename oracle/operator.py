"""ORACLE (test infrastructure only): the discrete Helmholtz operator.

Paper, section "Full waveform inversion in the space-frequency domain":
Eq. (2) is the constant-density Helmholtz equation
    -Laplace(u) - omega^2 m^2 (1 - j alpha) u = f,
with m = 1/c the real slowness and alpha the damping; Eq. (1) states that the
equation carries a first-order absorbing boundary condition; Eq. (3) writes
the discretised problem as B u = f.

Readings of what the paper leaves open (each listed in the design doc):

* Grid: nodes (iz, ix) at z = iz h, x = ix h, flat index iz*nx + ix; every
  edge of the rectangle absorbs. In 1D the single axis is x. Eq. (1) allows
  d = 3 as well: nodes (iz, iy, ix), flat index (iz*ny + iy)*nx + ix, every
  face of the box absorbing.
* Absorbing condition: du/dn + j omega m u = 0 on the boundary (n the outward
  normal, undamped wavenumber). Second-order centred differences; the ghost
  node beyond an edge is eliminated with the centred form of the condition.
* Each row is then multiplied by its control-volume weight w (the product of
  the axes' weights), with w_axis = 1/2 on the two end nodes of an axis and 1
  elsewhere. The result is
  the complex-symmetric matrix
      A = L / h^2 + (j omega / h) diag(g m) - omega^2 s diag(w m^2),
  where L is the real symmetric Neumann Laplacian whose coupling between two
  neighbours along one axis is the product of the other axes' weights, and g
  sums that product over the axis ends a node lies on.
  s = 1 - j alpha gives B; s = beta1 - j beta2 gives the shifted Laplacian M
  (same boundary term).
* A unit point source at node p is b = e_p / h^dim in this weighted system.

Variable density, Eq. (1) as printed: -div(rho grad u) - k^2 (1 - j alpha) u
= f with rho > 0 multiplying the flux and not the mass term (Eq. (2) is the
case rho = 1). Readings (listed in the design doc):

* the coupling of two neighbours is multiplied by the density on their
  common face, the mean (rho_p + rho_q) / 2 of the two nodes' densities;
* the absorbing condition is written for the flux, rho du/dn + j omega m
  sqrt(rho) u = 0: outgoing for the local wavenumber omega m / sqrt(rho) of
  the equation, and du/dn + j omega m u = 0 again at rho = 1. The boundary
  term of the matrix becomes (j omega / h) diag(g m sqrt(rho)).

With a constant density c this gives exactly c times the constant-density
matrix of the slowness m / sqrt(c).
"""

import numpy as np
import scipy.sparse as sp


def end_weights(n):
    """Control-volume weight along one axis: 1/2 at both end nodes, else 1."""
    w = np.ones(n)
    w[0] = 0.5
    w[-1] = 0.5
    return w


def stencil_parts(shape, rho=None):
    """Return (L, g, w) for a grid of the given shape (n,), (nz, nx) or
    (nz, ny, nx), axes in that order, the last one fastest in the flat order.

    L is the weighted Neumann Laplacian without the 1/h^2 factor (sparse,
    real, symmetric): two neighbours along an axis are coupled by the product
    of the other axes' weights (the face between their control volumes).
    g is the boundary-term weight: a node on an end of an axis gets that same
    product for each such end. w is the mass weight, the product of all the
    axes' weights. g and w are flattened in the grid's flat order. With a
    density rho (the grid's shape) every coupling is multiplied by the mean
    density of its two nodes.
    """
    shape = tuple(int(n) for n in shape)
    dim = len(shape)
    size = int(np.prod(shape))
    ws = [end_weights(n) for n in shape]
    idx = np.arange(size).reshape(shape)
    ps, qs, cs = [], [], []
    g = np.zeros(shape)
    for a in range(dim):
        face = np.ones(shape)
        for b in range(dim):
            if b != a:
                face = face * ws[b].reshape([-1 if i == b else 1 for i in range(dim)])
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[a], hi[a] = slice(0, -1), slice(1, None)
        ps.append(idx[tuple(lo)].ravel())
        qs.append(idx[tuple(hi)].ravel())
        cs.append(face[tuple(lo)].ravel())
        for end in (0, -1):
            sel = [slice(None)] * dim
            sel[a] = end
            g[tuple(sel)] += face[tuple(sel)]
    p, q, c = np.concatenate(ps), np.concatenate(qs), np.concatenate(cs)
    if rho is not None:
        rf = np.asarray(rho, dtype=np.float64).ravel()
        c = c * 0.5 * (rf[p] + rf[q])
    w = ws[0]
    for b in range(1, dim):
        w = np.multiply.outer(w, ws[b])
    off = sp.coo_matrix((np.concatenate([-c, -c]),
                         (np.concatenate([p, q]), np.concatenate([q, p]))),
                        shape=(size, size))
    deg = np.bincount(p, weights=c, minlength=size) + \
        np.bincount(q, weights=c, minlength=size)
    L = (off + sp.diags(deg)).tocsr()
    return L, g.ravel(), np.asarray(w).ravel()


def helmholtz_matrix(m, h, omega, s, rho=None):
    """A = L/h^2 + (j omega/h) diag(g m) - omega^2 s diag(w m^2), CSR complex128.

    m: slowness, shape (n,), (nz, nx) or (nz, ny, nx). s: complex mass shift;
    s = 1 - j alpha is the operator B of Eq. (2)-(3), s = beta1 - j beta2 the
    shifted Laplacian M. rho: density of Eq. (1) (None: 1), which weights the
    couplings by face densities and the boundary term by sqrt(rho).
    """
    m = np.asarray(m, dtype=np.float64)
    L, g, w = stencil_parts(m.shape, rho)
    mf = m.ravel()
    gm = g * mf if rho is None else g * mf * np.sqrt(np.asarray(rho, dtype=np.float64).ravel())
    diag = 1j * omega * gm / h - omega ** 2 * complex(s) * w * mf ** 2
    return (L.astype(np.complex128) / h ** 2 + sp.diags(diag)).tocsr()


def operator_B(m, h, omega, alpha, rho=None):
    """The damped Helmholtz operator B of Eq. (2)-(3) (Eq. (1) with a density rho)."""
    return helmholtz_matrix(m, h, omega, 1.0 - 1j * alpha, rho)


def operator_M(m, h, omega, beta1, beta2, rho=None):
    """The shifted-Laplace operator M = -Laplace - (beta1 - j beta2) omega^2 m^2
    (-div(rho grad) for the flux with a density rho)."""
    return helmholtz_matrix(m, h, omega, beta1 - 1j * beta2, rho)


def effective_slowness(m, rho=None):
    """m / sqrt(rho): the slowness the density-weighted equation propagates
    with (its local wavenumber is omega m / sqrt(rho))."""
    m = np.asarray(m, dtype=np.float64)
    return m if rho is None else m / np.sqrt(np.asarray(rho, dtype=np.float64))


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
