"""The oracle's public entry point: setup + V-ASMG-preconditioned CG solve.

Test infrastructure only (see the package header).

Setup (Section 3, setup step): assemble the P1 stiffness matrix (Section 2),
eliminate the fully fixed vertices, build the region tree and levels
(Section 3.1), the prolongations (Section 3.2), the Galerkin coarse operators,
the colourings and the coarsest Cholesky factor. Solve (Section 2.2,
Algorithm 2) with one V-cycle (Algorithm 3, recursive) as the preconditioner.

Options mirror the C library's: leaf_capacity (4 in 2D as in Section 3.1.1; 8 in
3D), n_pre/n_post sweeps, precision ('fp64' or 'fp32' V-cycle), tree vertices
('all' mesh vertices, as in Section 3.1.1, or only 'free' ones),
coarsest_max_dofs (0 = coarsen to the root region, as in Section 3.1.2),
smoother order ('colored' or the paper's 'lex'), colour blocks ('auto' or
'off': every cell its own colour block).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import fem, hierarchy, tree
from .pcg import pcg
from .smoother import BlockJacobi, ColoredGS, LexGS
from .vcycle import VCycle


@dataclass
class OracleOptions:
    leaf_capacity: int = 0          # 0 -> 4 (2D) / 8 (3D)
    n_pre: int = 1
    n_post: int = 1
    precision: str = "fp64"         # 'fp64' | 'fp32' (V-cycle only)
    tree_vertices: str = "all"      # 'all' | 'free'
    coarsest_max_dofs: int = 0
    max_iters: int = 10000
    smoother: str = "colored"       # 'colored' | 'lex' | 'jacobi'
    color_blocks: str = "off"       # 'off' | 'auto' (oracle/hierarchy.py block_steps)
    flexible: bool = False
    cycle: str = "V"                # 'V' | 'W' | 'additive' (oracle/vcycle.py)


class Oracle:
    def __init__(self, coords, elems, E, nu, fixed, opts: OracleOptions | None = None):
        t0 = time.perf_counter()
        self.opts = opts = opts or OracleOptions()
        coords = np.asarray(coords, dtype=np.float64)
        elems = np.asarray(elems, dtype=np.int64)
        nvtx, d = coords.shape
        self.d = d
        self.n_vertices = nvtx
        E = np.broadcast_to(np.asarray(E, dtype=np.float64), (elems.shape[0],))
        nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (elems.shape[0],))
        cap = opts.leaf_capacity or (4 if d == 2 else 8)
        self.capacity = cap

        # Section 2: stiffness matrix, Dirichlet elimination (fully fixed vertices
        # eliminated, fixed components of the other vertices as identity rows)
        self.K = fem.assemble(coords, elems, E, nu)
        self.free = fem.free_vertices(fixed)
        if self.free.size == 0:
            raise ValueError("no free vertices")
        cmask0 = fem.constrained_dofs(fixed, self.free)
        A0 = fem.restrict_free(self.K, self.free, d, cmask0)
        S0 = fem.fine_pattern(elems, self.free, nvtx)

        # Section 3.1 / 3.2: tree, levels, prolongations
        if opts.tree_vertices == "all":
            tree_idx = np.arange(nvtx)
        elif opts.tree_vertices == "free":
            tree_idx = self.free
        else:
            raise ValueError(opts.tree_vertices)
        pos_in_tree = np.full(nvtx, -1)
        pos_in_tree[tree_idx] = np.arange(tree_idx.size)
        self.levels = tree.build_levels(coords[tree_idx], coords[self.free],
                                        pos_in_tree[self.free], cap)

        # Section 3 setup step: Galerkin operators and structural patterns; the
        # constrained DOFs of each level (none without partial constraints)
        A = [A0]
        S = [S0]
        cm = [cmask0]
        for P in self.levels.prolong:
            cm.append(hierarchy.coarse_constraints(P, d, cm[-1]))
            A.append(hierarchy.galerkin(A[-1], P, d, cm[-2], cm[-1]))
            S.append(hierarchy.galerkin_pattern(S[-1], P))
        P_list = list(self.levels.prolong)
        # optional truncation: first level small enough becomes the coarsest
        if opts.coarsest_max_dofs > 0:
            for l, Al in enumerate(A):
                if Al.shape[0] <= opts.coarsest_max_dofs:
                    A, S, P_list, cm = A[:l + 1], S[:l + 1], P_list[:l], cm[:l + 1]
                    break
        self.A = A
        self.S = S
        self.P = P_list
        self.cmask = cm
        self.L = len(A) - 1
        # Gauss-Seidel visiting order: cells (single vertices on the fine level,
        # lattice cells of twice the finest spacing on coarse levels) grouped
        # into colour blocks, which are coloured
        self.cells, self.blocks, self.block_colors, self.cell_colors, self.colors = [], [], [], [], []
        self.block_steps = []
        for l in range(self.L):
            n = A[l].shape[0] // d
            if l == 0:
                cell_of = block_of = np.arange(n)
                bkeys, steps = None, 1
            else:
                keys = self.levels.level_keys(l)
                dstar = int(self.levels.regions[l - 1][0].max())
                h = int(tree.side_of(dstar))
                cell_of, ckeys = hierarchy.cell_partition(keys, 2 * h)
                steps = hierarchy.block_steps(hierarchy.coupling_reach(S[l], keys, h), d,
                                              opts.color_blocks)
                if steps == 2:
                    block_of, bkeys = cell_of, ckeys
                else:
                    block_of, bkeys = hierarchy.cell_partition(keys, steps * h)
            nblock = int(block_of.max()) + 1 if n else 0
            G = hierarchy.cell_graph(S[l], block_of, nblock)
            bc = hierarchy.choose_cell_coloring(G, bkeys)
            self.cells.append(cell_of)
            self.blocks.append(block_of)
            self.block_colors.append(bc)
            self.block_steps.append(steps)
            ncell = int(cell_of.max()) + 1 if n else 0
            cc = np.zeros(ncell, dtype=np.int64)
            cc[cell_of] = bc[block_of]
            self.cell_colors.append(cc)
            self.colors.append(bc[block_of])
        self.coarsest = hierarchy.CoarsestSolver(A[self.L])
        self.setup_seconds = time.perf_counter() - t0
        self._vcycles = {}

    # ------------------------------------------------------------------
    def vcycle(self, precision: str | None = None, smoother: str | None = None,
               cycle: str | None = None) -> VCycle:
        precision = precision or self.opts.precision
        smoother = smoother or self.opts.smoother
        cycle = cycle or self.opts.cycle
        key = (precision, smoother, cycle)
        if key not in self._vcycles:
            dt = np.float32 if precision == "fp32" else np.float64
            if smoother == "colored":
                sm = [self.gs(l, dt) for l in range(self.L)]
            elif smoother == "lex":
                sm = [LexGS(self.A[l], self.d, dt) for l in range(self.L)]
            elif smoother == "jacobi":
                sm = [BlockJacobi(self.A[l], self.d, dt, self.cmask[l]) for l in range(self.L)]
            else:
                raise ValueError(smoother)
            self._vcycles[key] = VCycle(self.A, self.P, sm, self.coarsest, self.d,
                                        self.opts.n_pre, self.opts.n_post, dt, cycle,
                                        cmask=self.cmask)
        return self._vcycles[key]

    def gs(self, l: int, dtype=np.float64) -> ColoredGS:
        """The coloured Gauss-Seidel sweeps of level l (the order the GPU uses)."""
        return ColoredGS(self.A[l], self.d, self.blocks[l], self.block_colors[l], dtype,
                         cell_of=self.cells[l])

    def apply_precond(self, r_free: np.ndarray, precision=None, smoother=None) -> np.ndarray:
        """z = B r on free DOFs (vertex-major, fine canonical order)."""
        vc = self.vcycle(precision, smoother)
        return vc.apply(r_free).astype(np.float64)

    def to_free(self, F: np.ndarray) -> np.ndarray:
        """[n_vertices, d] -> free-DOF vector (vertex-major); fixed components of
        the kept vertices are 0 (their entries of F are ignored)."""
        v = np.asarray(F, dtype=np.float64)[self.free].ravel().copy()
        v[self.cmask[0]] = 0.0
        return v

    def from_free(self, x: np.ndarray) -> np.ndarray:
        out = np.zeros((self.n_vertices, self.d))
        out[self.free] = x.reshape(-1, self.d)
        return out

    def solve(self, F: np.ndarray, rtol: float = 1e-6, precision=None, smoother=None,
              precond: str = "vasmg", max_iters: int | None = None, x0=None):
        """PCG (Algorithm 2). F and the result are [n_vertices, d]; fixed DOFs of F
        are ignored and 0 in the result. precond: 'vasmg' | 'jacobi' | 'none'."""
        b = self.to_free(F)
        if precond == "vasmg":
            vc = self.vcycle(precision, smoother)
            M = lambda r: vc.apply(r).astype(np.float64)  # noqa: E731
        elif precond == "jacobi":
            dinv = 1.0 / self.A[0].diagonal()
            M = lambda r: dinv * r  # noqa: E731
        elif precond == "none":
            M = lambda r: r.copy()  # noqa: E731
        else:
            raise ValueError(precond)
        t0 = time.perf_counter()
        x, info = pcg(self.A[0], b, M, rtol, max_iters or self.opts.max_iters,
                      None if x0 is None else self.to_free(x0), self.opts.flexible)
        info["solve_seconds"] = time.perf_counter() - t0
        return self.from_free(x), info

    def direct_solve(self, F: np.ndarray) -> np.ndarray:
        from scipy.sparse.linalg import spsolve
        b = self.to_free(F)
        return self.from_free(spsolve(self.A[0].tocsc(), b))

    def level_stats(self):
        out = []
        for l, A in enumerate(self.A):
            nv = A.shape[0] // self.d
            nb = self.S[l].nnz
            out.append(dict(level=l, n_vertices=nv, n_dofs=A.shape[0], n_blocks=int(nb),
                            n_colors=int(self.colors[l].max() + 1) if l < self.L else 0,
                            n_cells=int(self.cell_colors[l].size) if l < self.L else 0,
                            n_color_blocks=int(self.block_colors[l].size) if l < self.L else 0,
                            block_steps=self.block_steps[l] if l < self.L else 0))
        return out
