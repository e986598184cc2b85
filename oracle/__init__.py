"""CPU oracle for the V-ASMG-preconditioned CG solve (arXiv 2505.09064).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
anything in this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code with the HIP library; the only
common dependency is the seeded input generator package ``workloads``.

It is a plain, slow, step-by-step FP64 NumPy/SciPy implementation of what the
paper's method computes:

  fem.py        P1 linear-elasticity stiffness matrix (Section 2, problem and
                weak form, Lame constants, block matrix form of the system)
  tree.py       auxiliary region-tree, coarse levels and bilinear/trilinear
                prolongation weights (Section 3.1.1 Steps 1-4, Section 3.1.2,
                Section 3.2)
  hierarchy.py  Galerkin coarse operators R A P with R = P^T (Section 3,
                two-level setup step), greedy multicolouring, coarsest
                Cholesky factor (Section 3, solving step)
  smoother.py   Gauss-Seidel sweeps (Section 2.1, Algorithm 1), in the
                multicolour order the GPU uses and in the paper's lexicographic
                component-major order
  vcycle.py     the V-cycle preconditioner (Section 3, Algorithm 3 applied
                recursively)
  pcg.py        preconditioned conjugate gradients (Section 2.2, Algorithm 2)
  solver.py     the Oracle class tying the pieces together

Parity status of each part is listed in the module headers; every function
cites the passage of the paper it follows.
"""
from .solver import Oracle, OracleOptions  # noqa: F401
