"""MI355X-native V-ASMG-preconditioned CG for P1 linear elasticity (arXiv 2505.09064).

The solver is libvasmg.so (C ABI in include/vasmg.h): host setup of the
region-tree hierarchy and hand-written HIP kernels for gfx950 for the whole
solve phase. This package is its thin Python binding.
"""
from .vasmg import (  # noqa: F401
    EXPORTED, FP32_PRECOND, FP64, PRECOND_JACOBI, PRECOND_NONE, PRECOND_VASMG, TREE_ALL,
    TREE_FREE, Options, SolveInfo, Solver, VasmgError, default_options, last_error, lib,
)
