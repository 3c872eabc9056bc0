"""ORACLE (test infrastructure only): receiver sampling and the misfit J(m).

Eq. (4): J(m) = || u_obs - u_cal(m) ||_2^2 + (regularisation weight) |m|_2^2,
summed over shots, receivers and frequencies. The paper names the
regularisation weight alpha, the same letter as the damping of Eq. (2); here
it is lam. The regulariser is the plain squared norm of the slowness values
(no cell-area weight). Receivers sample the wavefield at grid nodes (no
interpolation).
"""

import numpy as np


def sample(u, rec_nodes):
    """d_cal = P u: wavefield values at the receiver nodes (flat indices)."""
    return np.asarray(u)[..., np.asarray(rec_nodes, dtype=np.int64)]


def misfit(d_obs, d_cal, m, lam):
    """J = sum |d_obs - d_cal|^2 + lam * sum m^2."""
    diff = np.asarray(d_obs, dtype=np.complex128) - np.asarray(d_cal, dtype=np.complex128)
    return float(np.sum(diff.real ** 2 + diff.imag ** 2) + lam * np.sum(np.asarray(m, float) ** 2))
