"""Galerkin coarse operators, multicolouring and the coarsest factor (oracle).

Test infrastructure only (see the package header).

Follows Section 3 (two-level setup step): R = P^T and A^c = R A P, applied
level by level, with P = P_scalar (x) I_d because the interpolation weight is the
same for every displacement component (Section 3.2). The coarsest system is
solved directly (Section 3, solving step; Section 4 takes B_0 = A_0^{-1}); here
by a dense FP64 Cholesky factorisation.

The multicolouring is not in the paper (its Gauss-Seidel is sequential); it
fixes the order in which the GPU's parallel Gauss-Seidel visits the vertices.
On the fine level every vertex is its own cell; on coarse levels vertices are
grouped into lattice cells of twice the level's finest spacing (at most 2^d
vertices). Cells are coloured greedily (first fit) on the cell adjacency graph
derived from the structural block pattern; the sweep visits colours in order,
the cells of a colour in any order (they are uncoupled) and the vertices of a
cell one after the other in canonical order.

Pins (tests/test_oracle_solver.py, test_galerkin_spd_and_rigid_modes and
test_cells_and_coloring): A_l symmetric positive definite, positive diagonal,
coarse operators annihilate the interpolated rigid-body modes of the
unconstrained operator, colouring validity.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def block_prolongation(P: sp.csr_matrix, d: int) -> sp.csr_matrix:
    """P (x) I_d in vertex-major DOF order (same weight for every component)."""
    return sp.kron(P, sp.identity(d, format="csr"), format="csr")


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix, d: int) -> sp.csr_matrix:
    """A_{l+1} = P_l^T A_l P_l (Section 3, equations (R) and (Ac))."""
    Pb = block_prolongation(P, d)
    Ac = (Pb.T @ A @ Pb).tocsr()
    Ac.sort_indices()
    return Ac


def galerkin_pattern(S: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Structural vertex pattern of P^T A P from the pattern of A (all values >0)."""
    Pp = P.copy()
    Pp.data = np.ones_like(Pp.data)
    return (Pp.T @ S @ Pp).tocsr()


def greedy_coloring(S: sp.csr_matrix) -> np.ndarray:
    """First-fit colouring in index order: vertex i takes the smallest colour not
    held by an already-coloured neighbour (diagonal ignored)."""
    S = S.tocsr()
    n = S.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    indptr, indices = S.indptr, S.indices
    for i in range(n):
        nb = indices[indptr[i]:indptr[i + 1]]
        used = color[nb]
        used = used[used >= 0]
        if used.size == 0:
            color[i] = 0
            continue
        mark = np.zeros(used.max() + 2, dtype=bool)
        mark[used] = True
        color[i] = int(np.argmin(mark))
    return color


def greedy_coloring_in_order(S: sp.csr_matrix, order: np.ndarray) -> np.ndarray:
    """First-fit colouring visiting the vertices in ``order``."""
    S = S.tocsr()
    n = S.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    indptr, indices = S.indptr, S.indices
    for i in order:
        nb = indices[indptr[i]:indptr[i + 1]]
        used = color[nb]
        used = used[used >= 0]
        if used.size == 0:
            color[i] = 0
            continue
        mark = np.zeros(used.max() + 2, dtype=bool)
        mark[used] = True
        color[i] = int(np.argmin(mark))
    return color


def cell_partition(keys: np.ndarray, cell_side: int):
    """Groups lattice vertices into cells of side ``cell_side`` (key // cell_side).

    Returns (cell_of_vertex, cell_keys) with cells numbered in canonical (z, y, x)
    order of their cell keys. Vertices keep their canonical order inside a cell.
    """
    ck = keys // cell_side
    d = keys.shape[1]
    uniq, inv = np.unique(ck[:, ::-1], axis=0, return_inverse=True)
    return inv.ravel().astype(np.int64), uniq[:, ::-1].copy()


def cell_graph(S: sp.csr_matrix, cell_of: np.ndarray, n_cells: int) -> sp.csr_matrix:
    """Cells are adjacent when any of their vertices are (structural pattern)."""
    C = S.tocoo()
    G = sp.csr_matrix((np.ones(C.nnz), (cell_of[C.row], cell_of[C.col])), shape=(n_cells, n_cells))
    G.sum_duplicates()
    return G


def choose_cell_coloring(G: sp.csr_matrix, cell_keys: np.ndarray | None) -> np.ndarray:
    """Greedy first-fit colouring of the cell graph with the fewest colours among
    three visiting orders: canonical, then lattice classes (cell key mod 2) and
    (cell key mod 3) in class order (canonical inside a class). Ties keep the
    earlier order. Without lattice keys only the canonical order is used."""
    n = G.shape[0]
    best = greedy_coloring_in_order(G, np.arange(n))
    if cell_keys is None:
        return best
    d = cell_keys.shape[1]
    for q in (2, 3):
        cls = np.zeros(n, dtype=np.int64)
        for a in range(d):
            cls += (cell_keys[:, a] % q) * q ** a
        order = np.lexsort((np.arange(n), cls))
        cand = greedy_coloring_in_order(G, order)
        if cand.max() < best.max():
            best = cand
    return best


def coloring_is_valid(S: sp.csr_matrix, color: np.ndarray) -> bool:
    C = S.tocoo()
    off = C.row != C.col
    return bool(np.all(color[C.row[off]] != color[C.col[off]]))


class CoarsestSolver:
    """Direct solve of the coarsest system A_L e = b by a dense FP64 Cholesky factor.

    A squared pivot at or below 1e-12 times the largest diagonal entry is
    treated as a singular operator (e.g. no fixed DOFs: the rigid-body modes are
    linear, so they survive on every level)."""

    def __init__(self, A: sp.csr_matrix):
        dense = A.toarray()
        try:
            self.c = sla.cho_factor(dense, lower=True)
        except np.linalg.LinAlgError as exc:
            raise np.linalg.LinAlgError("coarsest operator is not positive definite") from exc
        # a pivot below 1e-12 * max(diag A) is taken as numerically singular
        piv = np.diag(self.c[0]) ** 2
        if piv.min() <= 1e-12 * np.diag(dense).max():
            raise np.linalg.LinAlgError("coarsest operator is numerically singular")
        self.n = dense.shape[0]

    def solve(self, b: np.ndarray) -> np.ndarray:
        return sla.cho_solve(self.c, np.asarray(b, dtype=np.float64))
