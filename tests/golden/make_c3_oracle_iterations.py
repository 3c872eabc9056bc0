"""Write c3_oracle_iterations.json: the oracle's own BiCGSTAB iteration counts
(tol 1e-8, V(2,2) shifted-Laplace (1, 0.5) preconditioner with the default
plan: LFA-planned levels and weights, and the coarsest level solved exactly
or, where its smallest kh is at least 2.5, smoothed by two damped-Jacobi
sweeps -- the solver library's default policy) on the 401 x 801 layered
model for three of its 64 surface shots at each of the frequencies 3, 5, 8
and 12 Hz. Calls only oracle/ (and the input generators).

Run from the repository root: python tests/golden/make_c3_oracle_iterations.py
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

SHOTS = (0, 31, 63)


def main():
    w = workloads.model_2d_layered()
    out = {"workload": w.name, "tol": 1e-8, "beta": [1.0, 0.5], "nu": [2, 2], "coarse_policy": "auto",
           "shots": list(SHOTS),
           "freqs": {}}
    for f in w.freqs:
        om = 2 * np.pi * f
        B = op.operator_B(w.m, w.h, om, w.alpha)
        L, wj = lfa.plan(w.shape, w.h, om, w.m.min(), w.m.max(), 1.0, 0.5)
        V = mg.VCycle(w.m, w.h, om, 1.0, 0.5, L, 2, 2, wj, coarse="auto")
        hc = w.h * 2.0 ** (L - 1)
        coarse = "jacobi" if om * hc * w.m.min() >= 2.5 else "exact"
        its = []
        t0 = time.perf_counter()
        for s in SHOTS:
            b = op.point_source(w.shape, w.h, [w.src[s]])
            _, it, rr, st = krylov.bicgstab(B, b, V, tol=1e-8, maxit=2000)
            assert st == krylov.CONVERGED, (f, s, st)
            its.append(int(it))
        secs = time.perf_counter() - t0
        out["freqs"][str(f)] = {"levels": L, "jacobi_w": wj, "coarse": coarse, "iterations": its,
                                "mean_iterations": float(np.mean(its))}
        print(f, L, wj, its, f"{secs:.1f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_iterations.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
