"""Plain FP64 CPU oracle for the shifted-Laplace preconditioned Helmholtz solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it. It shares no code, constant or table with the HIP library
under ``paper_1712_08743_amd/``; both sides receive the same seeded inputs from
the ``workloads`` package, which holds none of the method's arithmetic.

Source: N. Kazemi, "Application of shifted-Laplace preconditioners for
heterogenous Helmholtz equation -- part 2: Full waveform inversion"
(arXiv:1712.08743). Section "Full waveform inversion in the space-frequency
domain": Eq. (2) (constant-density Helmholtz equation with damping), Eq. (3)
(the discrete system B u = f), Eq. (4) (misfit), Eq. (7) (gradient).

Every floating-point quantity is float64 / complex128.

Modules
-------
operator    the discrete operator B (and the shifted Laplacian M) as a sparse
            matrix, and point sources                       -- Eq. (2), (3)
direct      sparse LU (SuperLU), an own banded LU, dense solve -- "LU
            factorization" used for observed data (Examples section)
multigrid   the geometric V-cycle that approximates M^-1   -- the
            preconditioner (Examples/Conclusion: shifted-Laplace operator)
krylov      right-preconditioned BiCGSTAB and GMRES(m)     -- "Krylov
            subspace ... GMRES" (section on FWI, Conclusion)
lfa         local Fourier analysis of damped Jacobi and the level/weight plan
misfit      receiver sampling and J(m)                      -- Eq. (4)
gradient    adjoint-state gradient, Born modelling and the Gauss-Newton
            operator                                       -- Eq. (7)-(9)
"""

from . import operator, direct, multigrid, krylov, lfa, misfit, gradient  # noqa: F401
