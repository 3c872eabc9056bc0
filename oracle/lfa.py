"""ORACLE (test infrastructure only): local Fourier analysis of damped Jacobi
on the shifted-Laplace operator, and the level / weight plan built on it.

For the interior stencil of h^2 M (dim axes), a Fourier mode with angles
theta has the Laplacian symbol l(theta) = sum_axes (2 - 2 cos theta_a) and the
mass symbol s q with s = beta1 - j beta2, q = (k h)^2, k = omega m. Damped
Jacobi multiplies the mode's error by 1 - w (l - s q) / (2 dim - s q). The
high-frequency modes (some |theta_a| >= pi/2) have l in [2, 4 dim]; since the
factor is affine in l, its largest modulus over them sits at l = 2 or
l = 4 dim. That largest modulus is the smoothing factor mu(kh).

The paper gives no multigrid; the plan below is this build's reading:

* levels: coarsen while every axis n satisfies (n - 1) even and
  (n - 1)/2 + 1 >= 3, unless a level count is requested;
* weight of smoothing level l: the largest w in WEIGHTS (not above the
  requested default) whose mu stays <= 1 at KH_SAMPLES evenly spaced kh
  between omega h_l min(m) and omega h_l max(m) (end points included); if no
  candidate qualifies, the one with the smallest worst-case mu (first on ties).
"""

import numpy as np

WEIGHTS = (0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2)
KH_SAMPLES = 65


def smoothing_factor(kh, beta1, beta2, w, dim=2):
    """mu(kh) = max over high-frequency modes of |1 - w (l - s q)/(2 dim - s q)|."""
    s = complex(beta1, -beta2)
    q = float(kh) ** 2
    den = 2 * dim - s * q

    def amp(l):
        return abs(1 - w * (l - s * q) / den)

    return max(amp(2.0), amp(4.0 * dim))


def smoothing_factor_sampled(kh, beta1, beta2, w, dim=2, n=129):
    """The same maximum taken by brute force over a grid of mode angles."""
    s = complex(beta1, -beta2)
    q = float(kh) ** 2
    t = np.linspace(-np.pi, np.pi, n)
    th = np.meshgrid(*([t] * dim), indexing="ij")
    hi = np.zeros(th[0].shape, dtype=bool)
    lsym = np.zeros(th[0].shape)
    for ta in th:
        hi |= np.abs(ta) >= np.pi / 2
        lsym += 2 - 2 * np.cos(ta)
    a = np.abs(1 - w * (lsym - s * q) / (2 * dim - s * q))
    return float(a[hi].max())


COARSE_TARGET = 512  # unknowns on the coarsest level a default plan aims at or below


def max_levels(shape):
    """Largest level count the grid allows: halve (n -> ceil(n / 2)) while
    every axis keeps at least 3 nodes."""
    L = 1
    cur = list(shape)
    while all(n >= 5 for n in cur):
        cur = [(n + 1) // 2 for n in cur]
        L += 1
    return L


def default_levels(shape):
    """Levels of a default plan: halve while the coarsest level has more than
    COARSE_TARGET unknowns and every axis keeps at least 3 nodes."""
    L = 1
    cur = list(shape)
    while int(np.prod(cur)) > COARSE_TARGET and all(n >= 5 for n in cur):
        cur = [(n + 1) // 2 for n in cur]
        L += 1
    return L


def plan(shape, h, omega, m_min, m_max, beta1, beta2, w_default=0.8, levels=0):
    """Return (levels, [w_0, ..., w_{L-2}]) for one frequency."""
    dim = len(shape)
    L = levels if levels > 0 else default_levels(shape)
    weights = []
    for l in range(L - 1):
        hl = h * 2.0 ** l
        lo, hi = omega * hl * m_min, omega * hl * m_max
        khs = [lo + (hi - lo) * i / (KH_SAMPLES - 1) for i in range(KH_SAMPLES)]
        best, best_mu = None, None
        chosen = None
        for w in WEIGHTS:
            if w > w_default + 1e-12:
                continue
            worst = max(smoothing_factor(kh, beta1, beta2, w, dim) for kh in khs)
            if worst <= 1.0:
                chosen = w
                break
            if best_mu is None or worst < best_mu:
                best, best_mu = w, worst
        weights.append(chosen if chosen is not None else best)
    return L, weights
