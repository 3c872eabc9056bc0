"""Gauss-Newton full waveform inversion driven by the library.

Each Gauss-Newton iteration (Eq. (9)) is one ``hz_gn_step`` on the current
model: the gradient of Eq. (7) from forward and adjoint solves, then CG on
the Gauss-Newton system with one Born and one adjoint batch per CG iteration
(three forward modellings per iteration in the paper's count). Two frequency
schedules, as in the paper's examples: all frequencies inverted together
(the 1D example) or groups from low to high, each group starting from the
previous group's model (the 2D example).
"""

import numpy as np


def invert(ctx, m0, h, freqs, alpha, src, rec, d_obs, lam, gn_iters, cg_iters, schedule="simultaneous",
           groups=None, step=1.0, m_true=None, **opt):
    """Run ``gn_iters`` Gauss-Newton iterations per frequency group.

    d_obs: complex [nfreq, nsrc, nrec] (numpy or torch) for ``freqs``;
    schedule "simultaneous" inverts all frequencies at once, "sequential"
    the groups in ``groups`` (lists of indices into freqs; default one
    frequency per group, low to high). ``step`` scales every update.
    Returns (m, history) with one record per iteration: group, J before the
    update, CG iterations, Krylov iterations of the forward solves and, when
    m_true is given, the relative model error after the update."""
    import torch
    # the model stays on the device: Eq. (9)'s update m + step dm is a device axpy
    m = torch.as_tensor(np.asarray(m0, dtype=np.float64) if not torch.is_tensor(m0) else m0,
                        dtype=torch.float64).to(ctx.device).clone()
    mt = None if m_true is None else torch.as_tensor(np.asarray(m_true, dtype=np.float64)).to(m.device)
    d_obs = torch.as_tensor(np.asarray(d_obs) if not torch.is_tensor(d_obs) else d_obs)
    order = np.argsort(freqs)
    if schedule == "simultaneous":
        groups = [list(range(len(freqs)))]
    elif groups is None:
        groups = [[int(i)] for i in order]
    history = []
    for gi, g in enumerate(groups):
        fr = [float(freqs[i]) for i in g]
        dg = d_obs[list(g)].contiguous()
        for _ in range(gn_iters):
            ctx.set_model(m, h)
            dm, J, it, info = ctx.gn_step(fr, alpha, src, rec, dg, lam, cg_iters, **opt)
            m.add_(dm, alpha=float(step))
            rec_ = {"group": gi, "freqs": fr, "J": J, "cg_iterations": it,
                    "krylov_iterations": int(sum(i[1] for i in info))}
            if mt is not None:
                rec_["model_error"] = float(torch.linalg.vector_norm(m - mt) / torch.linalg.vector_norm(mt))
            history.append(rec_)
    return m.cpu().numpy(), history
