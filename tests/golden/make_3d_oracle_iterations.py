"""Write l3d_oracle_iterations.json: the oracle's own BiCGSTAB iteration
counts (tol 1e-8, LFA-planned V(2,2) shifted-Laplace (1, 0.5) preconditioner
with the coarsest-level rule the library applies by default) on the layered
129 x 129 x 129 box (h = 20 m) for two of its eight surface shots at each of
the frequencies 3 and 5 Hz. Calls only oracle/ (and the input generators).

Run from the repository root: python tests/golden/make_3d_oracle_iterations.py
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import operator as op, multigrid as mg, krylov, lfa  # noqa: E402

SHOTS = (0, 7)


def main():
    w = workloads.model_3d_layered(129, 129, 129, h=20.0, nshots=8, freqs=(3.0, 5.0))
    out = {"workload": w.name, "h": w.h, "tol": 1e-8, "beta": [1.0, 0.5], "nu": [2, 2], "coarse": "auto",
           "shots": list(SHOTS), "freqs": {}}
    for f in w.freqs:
        om = 2 * np.pi * f
        B = op.operator_B(w.m, w.h, om, w.alpha)
        L, wj = lfa.plan(w.shape, w.h, om, float(w.m.min()), float(w.m.max()), 1.0, 0.5)
        V = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
        its = []
        t0 = time.perf_counter()
        for s in SHOTS:
            iz, iy, ix = w.src[s]
            b = op.point_source(w.shape, w.h, [(iz * w.shape[1] + iy) * w.shape[2] + ix])
            _, it, rr, st = krylov.bicgstab(B, b, V, tol=1e-8, maxit=2000)
            assert st == krylov.CONVERGED, (f, s, st)
            its.append(int(it))
        secs = time.perf_counter() - t0
        out["freqs"][str(f)] = {"levels": L, "jacobi_w": wj, "coarse": V.coarse, "iterations": its,
                                "mean_iterations": float(np.mean(its))}
        print(f, L, wj, V.coarse, its, f"{secs:.1f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "l3d_oracle_iterations.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
