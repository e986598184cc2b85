"""Gauss-Seidel sweeps (oracle).

Test infrastructure only (see the package header).

Point Gauss-Seidel of Section 2.1, Algorithm 1: each unknown i is replaced by
(f_i - sum_{j != i} a_ij u_j) / a_ii using the newest values of the unknowns
already visited. A V-cycle sweeps once forward before the coarse correction and
once in exactly the reverse order after it (Section 3, Step 2.5). Algorithm 1's
error-based exit is not used inside a V-cycle (a fixed number of sweeps).

Two visiting orders:
  * ``colored`` (the order the GPU uses): colours ascending, the colour blocks
    of a colour, the cells of a block and the vertices of a cell in canonical
    order, components ascending; the backward sweep is the exact reverse.
    Blocks of one colour are not coupled, so the same position of all of them
    can be updated at once for each component.
  * ``lex`` (the paper's order): all first components, then all second
    components, ... (the component-major unknown vector [U1; U2; ...] of
    Section 2), in vertex order; realised with triangular solves, since one
    forward sweep is x_new = (D - L)^{-1} (b + S x_old).

Pins (tests/test_oracle_solver.py, test_gauss_seidel_orders): a sweep equals a
literal element-by-element Algorithm 1 loop on small dense matrices; the
coloured sweep equals the lexicographic sweep of the colour-permuted matrix.
tests/test_oracle_precision.py: the float32 sweep equals a literal float32
point loop up to summation order and is not FP64; the Jacobi step in
test_oracle_solver.py, test_block_jacobi_smoother.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular


class ColoredGS:
    """Point GS over (colour, block, cell, vertex, component) on a vertex-major
    scalar CSR matrix.

    block_of[v] is the colour block of vertex v, block_color[k] the colour of
    block k, and cell_of[v] (optional; default: the block) the cell inside the
    block. The forward sweep visits colours ascending; blocks of one colour are
    uncoupled, so for each position p inside a block (cells ascending, then
    vertices ascending) and each component, the p-th vertices of all blocks of
    the colour are updated at once. The backward sweep is the exact reverse.
    """

    def __init__(self, A: sp.csr_matrix, d: int, block_of: np.ndarray, block_color: np.ndarray,
                 dtype=np.float64, cell_of: np.ndarray | None = None):
        self.d = d
        self.dtype = dtype
        A = A.astype(dtype).tocsr()
        diag = A.diagonal()
        n = A.shape[0] // d
        color = block_color[block_of]
        sub = block_of if cell_of is None else cell_of
        order = np.lexsort((np.arange(n), sub, block_of, color))   # colour, block, cell, vertex
        pos = np.zeros(n, dtype=np.int64)
        prev_block, k = -1, 0
        for v in order:
            k = k + 1 if block_of[v] == prev_block else 0
            pos[v] = k
            prev_block = block_of[v]
        ncol = int(color.max()) + 1 if n else 0
        self.parts = []          # per (colour, position): per component (rows, A[rows], a_ii)
        for c in range(ncol):
            for p in range(int(pos.max()) + 1):
                verts = np.flatnonzero((color == c) & (pos == p))
                if verts.size == 0:
                    continue
                comps = []
                for a in range(d):
                    rows = verts * d + a
                    comps.append((rows, A[rows].tocsr(), diag[rows]))
                self.parts.append(comps)

    def _update(self, part, b, x):
        rows, Ar, aii = part
        sigma = Ar @ x - aii * x[rows]            # sum over j != i of a_ij x_j
        x[rows] = (b[rows] - sigma) / aii

    def forward(self, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        x = x.astype(self.dtype, copy=True)
        for comps in self.parts:
            for part in comps:
                self._update(part, b, x)
        return x

    def backward(self, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        x = x.astype(self.dtype, copy=True)
        for comps in reversed(self.parts):
            for part in reversed(comps):
                self._update(part, b, x)
        return x


class LexGS:
    """Point GS in the paper's component-major order via triangular solves."""

    def __init__(self, A: sp.csr_matrix, d: int, dtype=np.float64):
        n = A.shape[0]
        nv = n // d
        v = np.arange(nv)
        self.perm = (v[None, :] * d + np.arange(d)[:, None]).ravel()   # cm position -> vm DOF
        Acm = A[self.perm][:, self.perm].astype(dtype).tocsr()
        self.low = sp.tril(Acm, format="csr")
        self.up = sp.triu(Acm, format="csr")
        self.strict_up = sp.triu(Acm, k=1, format="csr")
        self.strict_low = sp.tril(Acm, k=-1, format="csr")
        self.dtype = dtype

    def forward(self, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        xc = x[self.perm].astype(self.dtype)
        rhs = b[self.perm] - self.strict_up @ xc
        xn = spsolve_triangular(self.low, rhs, lower=True)
        out = np.empty_like(xc)
        out[self.perm] = xn
        return out.astype(self.dtype)

    def backward(self, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        xc = x[self.perm].astype(self.dtype)
        rhs = b[self.perm] - self.strict_low @ xc
        xn = spsolve_triangular(self.up, rhs, lower=False)
        out = np.empty_like(xc)
        out[self.perm] = xn
        return out.astype(self.dtype)


def jacobi_lambda_max(A: sp.csr_matrix, d: int, iters: int = 30,
                      cmask: np.ndarray | None = None) -> float:
    """Estimate of the largest eigenvalue of D^{-1} A (D = the d x d vertex blocks
    of A): power iteration from the all-ones vector on the unconstrained DOFs
    (0 on constrained ones, whose identity rows keep them 0), then the Rayleigh
    quotient v^T A v / v^T D v of the last iterate. FP64."""
    A = A.astype(np.float64).tocsr()
    n = A.shape[0]
    nv = n // d
    Dinv = _block_diag_inverse(A, d)
    v = np.ones(n)
    if cmask is not None:
        v[cmask] = 0.0
    for _ in range(iters):
        w = Dinv @ (A @ v)
        v = w / np.linalg.norm(w)
    D = sp.block_diag([A[k * d:(k + 1) * d, k * d:(k + 1) * d] for k in range(nv)], format="csr")
    return float(v @ (A @ v)) / float(v @ (D @ v))


def _block_diag_inverse(A: sp.csr_matrix, d: int) -> sp.csr_matrix:
    nv = A.shape[0] // d
    blocks = []
    for k in range(nv):
        blk = A[k * d:(k + 1) * d, k * d:(k + 1) * d].toarray()
        blocks.append(np.linalg.inv(blk))
    return sp.block_diag(blocks, format="csr")


class BlockJacobi:
    """Damped vertex-block Jacobi, one of the smoothers Section 4 names for S_h:
    x <- x + omega D^{-1} (b - A x), D = the d x d diagonal block of each vertex,
    omega = (4/3) / lambda_max(D^{-1} A) (the usual 2/3 when lambda_max = 2),
    lambda_max from jacobi_lambda_max. Forward and backward sweeps are the same
    step (Jacobi has no order). Pinned: the step equals the formula with dense
    matrices; omega * lambda_max < 2 for the exact lambda_max (the cycle stays
    symmetric positive definite)."""

    def __init__(self, A: sp.csr_matrix, d: int, dtype=np.float64, cmask=None):
        self.dtype = dtype
        self.lam = jacobi_lambda_max(A, d, cmask=cmask)
        self.omega = (4.0 / 3.0) / self.lam
        self.A = A.astype(dtype).tocsr()
        self.Dinv = _block_diag_inverse(A.astype(np.float64).tocsr(), d).astype(dtype)

    def forward(self, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        om = self.dtype(self.omega)
        return x + om * (self.Dinv @ (b - self.A @ x))

    backward = forward

