"""The V-ASMG V-cycle preconditioner (oracle).

Test infrastructure only (see the package header).

Section 3, Algorithm 3 (two-level V-cycle) applied recursively over the
region-tree levels (Section 3: the multi-level method is the recursion of the
two-level one). One application z = B r, from a zero initial guess:

  pre-smoothing   n_pre forward GS sweeps on A_l x = b           (Step 2.1)
  residual        r_l = b - A_l x                                 (Step 2.1)
  restriction     b_{l+1} = P_l^T r_l                              (Step 2.2)
  coarse solve    recursive cycle, or the direct solve at l = L   (Step 2.3)
  prolongation    x += P_l e_{l+1}                                 (Step 2.4)
  post-smoothing  n_post GS sweeps in the reverse order           (Step 2.5)

Algorithm 3's outer convergence loop is not used: a preconditioner application
is exactly one cycle.

Cycle modes (Section 3 names the V- and W-cycle; Section 4 defines the
preconditioner as B_h = S_h + Pi B_0 Pi^T):
  'V'         the recursion above, one coarse visit per level;
  'W'         two visits of level l+1 per visit of level l; the second starts from
              the first one's result (a cycle from the guess x0 returns
              x0 + B (b - A x0)); the coarsest level, solved exactly, once;
  'additive'  B r = S r + P_0 B_1 P_0^T r: S = the n_pre forward then n_post
              backward sweeps from zero on the fine level (symmetric
              Gauss-Seidel for V(1,1)), B_1 = one V-cycle of levels 1..L (the
              auxiliary space's solver), both applied to the same r.

In FP32 emulation (``dtype=np.float32``) the level matrices, weights and V-cycle
vectors are single precision; the coarsest right-hand side is cast to FP64,
solved in FP64 and cast back.

Pins (tests/test_oracle_solver.py, test_vcycle_closed_form_spd and the W-cycle
and additive tests): the dense operator of one cycle equals the closed form
B_l = Mbar^{-1} + (I - M^{-T} A_l) P_l B_{l+1} P_l^T (I - A_l M^{-1}) with
Mbar^{-1} = M^{-1} + M^{-T} - M^{-T} A_l M^{-1}; B is symmetric positive
definite; a one-level hierarchy gives B = A^{-1}. FP32 emulation
(tests/test_oracle_precision.py): every stored operator, weight and smoother
matrix is float32, the coarsest solve is FP64 (bitwise the rounded FP64 direct
solve on a one-level hierarchy), and the cycle sits between 1e-9 and 1e-5 of
the FP64 cycle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .hierarchy import masked_prolongation


class VCycle:
    def __init__(self, A_levels, P_levels, smoothers, coarsest, d: int,
                 n_pre: int = 1, n_post: int = 1, dtype=np.float64, cycle: str = "V",
                 cmask=None):
        """A_levels[0..L], P_levels[0..L-1] (scalar), smoothers[0..L-1], coarsest
        solver; cmask[l]: constrained DOFs of level l (zero prolongation rows)."""
        if cycle not in ("V", "W", "additive"):
            raise ValueError(cycle)
        self.cycle = cycle
        self.L = len(A_levels) - 1
        self.dtype = dtype
        self.A = [A.astype(dtype).tocsr() for A in A_levels]
        self.Pb = [masked_prolongation(P, d, None if cmask is None else cmask[l]).astype(dtype).tocsr()
                   for l, P in enumerate(P_levels)]
        self.PbT = [Pb.T.tocsr() for Pb in self.Pb]
        self.smoothers = smoothers
        self.coarsest = coarsest
        self.n_pre = n_pre
        self.n_post = n_post

    def apply(self, r: np.ndarray) -> np.ndarray:
        r = np.asarray(r).astype(self.dtype)
        if self.cycle == "additive" and self.L > 0:
            S = self.smoothers[0]
            z = np.zeros_like(r)
            for _ in range(self.n_pre):
                z = S.forward(r, z)
            for _ in range(self.n_post):
                z = S.backward(r, z)
            e1 = self._cycle(1, self.PbT[0] @ r, None, "V")
            return z + self.Pb[0] @ e1
        return self._cycle(0, r, None, self.cycle)

    def _cycle(self, l: int, b: np.ndarray, x0, mode: str) -> np.ndarray:
        if l == self.L:
            return self.coarsest.solve(b.astype(np.float64)).astype(self.dtype)
        S = self.smoothers[l]
        x = np.zeros_like(b) if x0 is None else x0.copy()
        for _ in range(self.n_pre):
            x = S.forward(b, x)
        r = b - self.A[l] @ x
        bc = self.PbT[l] @ r
        ec = self._cycle(l + 1, bc, None, mode)
        if mode == "W" and l + 1 < self.L:
            ec = self._cycle(l + 1, bc, ec, mode)
        x = x + self.Pb[l] @ ec
        for _ in range(self.n_post):
            x = S.backward(b, x)
        return x


def dense_operator(apply, n: int) -> np.ndarray:
    """Dense matrix of a linear map, column by column (small problems only)."""
    B = np.empty((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        B[:, j] = apply(e)
    return B


def sparse_identity_like(n: int):
    return sp.identity(n, format="csr")
