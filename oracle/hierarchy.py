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
vertices), and cells into colour blocks (block_steps: 3D levels whose
couplings reach 3 or 4 lattice steps take blocks of 4 steps, up to 8 cells;
otherwise a block is one cell). Blocks are coloured greedily (first fit) on
the block adjacency graph derived from the structural block pattern; the sweep
visits colours in order, the blocks of a colour in any order (they are
uncoupled), the cells of a block in canonical order and the vertices of a cell
in canonical order.

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


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix, d: int, cmask: np.ndarray | None = None,
             cmask_next: np.ndarray | None = None) -> sp.csr_matrix:
    """A_{l+1} = P_l^T A_l P_l (Section 3, equations (R) and (Ac)). With
    constrained DOFs (cmask, see masked_prolongation) the block prolongation's
    rows of the level's fixed components are zero, and every coarse DOF whose
    column is then empty (cmask_next) gets an identity row and column."""
    Pb = block_prolongation(P, d) if cmask is None else masked_prolongation(P, d, cmask)
    Ac = (Pb.T @ A @ Pb).tocsr()
    if cmask_next is not None and cmask_next.any():
        Ac = (Ac + sp.diags(cmask_next.astype(np.float64))).tocsr()
    Ac.sort_indices()
    return Ac


def masked_prolongation(P: sp.csr_matrix, d: int, cmask: np.ndarray) -> sp.csr_matrix:
    """P (x) I_d with zero rows at the level's constrained DOFs (cmask)."""
    Pb = block_prolongation(P, d)
    if cmask is None or not cmask.any():
        return Pb
    return (sp.diags((~cmask).astype(np.float64)) @ Pb).tocsr()


def coarse_constraints(P: sp.csr_matrix, d: int, cmask: np.ndarray) -> np.ndarray:
    """Constrained DOFs of the next level: a coarse component is constrained when
    every fine vertex interpolating from that coarse vertex has the component
    fixed (its column of the masked prolongation is empty)."""
    Pm = masked_prolongation(P, d, cmask)
    nnz = np.asarray((abs(Pm) > 0).sum(axis=0)).ravel()
    return nnz == 0


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


def coupling_reach(S: sp.csr_matrix, keys: np.ndarray, h: int) -> int:
    """Largest per-axis lattice distance, in steps of h, between two coupled
    vertices of a lattice level (structural pattern S, integer keys)."""
    C = S.tocoo()
    if C.nnz == 0:
        return 0
    return int(np.abs(keys[C.row] - keys[C.col]).max() // h)


def block_steps(reach: int, d: int, mode: str) -> int:
    """Side, in lattice steps, of the colour blocks of a 3D lattice level.

    Cells of side 2 steps are grouped into colour blocks: a colour is given to
    a block, and a sweep visits the cells of a block one after the other. Two
    blocks of side s whose indices differ by 2 along an axis are at least s + 1
    steps apart, so when the coupling reach is at most s only neighbouring
    blocks couple and 2^d colours suffice. Side 4 (up to 8 cells) is used when
    the reach is 3 or 4 steps ('auto', 3D only); otherwise a block is one cell."""
    if mode == "off" or d != 3:
        return 2
    if mode != "auto":
        raise ValueError(mode)
    return 4 if 2 < reach <= 4 else 2


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
