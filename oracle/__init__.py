"""Plain, slow FP64 CPU oracle for the phase-field fracture Newton/GMG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1902_08112_amd``); the only module both sides read is
``workloads`` (seeded synthetic inputs, no method arithmetic).

Every routine follows the paper (Jodlbauer, Langer, Wick, "Matrix-free
multigrid solvers for phase-field fracture problems", arXiv:1902.08112) by the
plainest route: dense element matrices by Gauss quadrature, assembled SciPy
CSR, SpMV, textbook Chebyshev / CG-Lanczos / V-cycle / FGMRES.

Modules
  fe      reference element, quadrature, uniform level meshes        (Sec. 2.4)
  model   residual A(U), Jacobian G(U), lumped mass, assembly        (Sec. 2.3, eq. semilinear; Sec. 3.1)
  mg      injection, transfers, diagonal, Chebyshev, V-cycle         (Sec. 3.2, Sec. 4.2)
  krylov  CG-Lanczos eigenvalue estimate, FGMRES                     (Sec. 3.2.1, Sec. 5)
  newton  one primal-dual active-set Newton step                     (Sec. 3.1, Algorithm 1)
  rng     SplitMix64 counter-based generator (start vectors)

Parity status of each function is stated in its docstring; a function with no
independent pin says "parity unpinned".
"""
