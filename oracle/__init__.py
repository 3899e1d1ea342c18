"""Plain FP64 CPU oracle for the L-sweeps hot path (arXiv:1909.01467).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its C
ABI or the Python binding) may import, call or link anything in this package;
only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the HIP path: it has its own discretisation, its
own domain partition, its own trace bookkeeping and its own Krylov solver.

Modules
  discretization  App. A: PML profile, symmetric PML operator, normal extension
  direct          the exact solve u = A^-1 b (banded LU, SuperLU, dense)
  lsweep          Alg. Scenario3 of App. C, run literally and sequentially
  lsweep3d        the same over a beam CDD of a 3D box (7-point operator)
  scenario4       Sec. 2.1 scenario 4: four shifted CDDs and a partition of unity
  fgmres          right-preconditioned flexible GMRES (Sec. 3, Phase 3)
  gradient        FWI misfit and its adjoint-state gradient (Sec. 1 motivation)

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
