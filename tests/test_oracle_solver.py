"""Pins of the oracle's hierarchy, Gauss-Seidel, V-cycle and PCG.

  * Galerkin operators (Section 3, equations (R), (Ac)): symmetric positive
    definite after the boundary conditions, positive diagonal, and for the
    unconstrained operator they annihilate the interpolated rigid-body modes.
  * Gauss-Seidel cells, colour blocks and colouring: cells are lattice blocks of
    at most 2^d vertices, colour blocks whole cells on a lattice of 2 or 4 steps
    (4 only where the couplings reach 3 or 4 steps, so that 2^d colours
    suffice), coupled vertices of different colour blocks never share a colour.
  * Gauss-Seidel (Section 2.1, Algorithm 1): equals a literal element-by-element
    loop in the same unknown order; one forward sweep from zero equals a
    lower-triangular solve; backward is the exact reverse order.
  * V-cycle (Algorithm 3, recursive): its dense operator equals the closed-form
    symmetric multigrid recursion, is symmetric positive definite; with the
    fine level as the coarsest, B = A^{-1}.
  * PCG (Algorithm 2): error within kappa * rtol of a dense solve; unpreconditioned
    CG within n iterations; iteration counts stay flat under refinement
    (Theorem 3: kappa(B A) bounded).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Oracle, OracleOptions, fem, hierarchy, tree
from oracle.pcg import pcg
from oracle.smoother import ColoredGS, LexGS
from oracle.vcycle import dense_operator
from workloads import manufactured_mesh, small2d, small3d


def _tiny(dim, **kw):
    if dim == 2:
        return small2d(7, seed=1, **kw)
    return small3d(4, seed=2, **kw)


@pytest.mark.parametrize("dim", [2, 3])
def test_galerkin_spd_and_rigid_modes(dim):
    m = _tiny(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    for A in o.A:
        Ad = A.toarray()
        assert np.abs(Ad - Ad.T).max() <= 1e-13 * np.abs(Ad).max()
        assert np.all(np.diag(Ad) > 0)
        assert np.linalg.eigvalsh(Ad)[0] > 0
    # unconstrained operator: coarse operators annihilate interpolated rigid modes
    from oracle import tree
    K = fem.assemble(m.coords, m.elems, 1.0, 0.3)
    allv = np.arange(m.n_vertices)
    lv = tree.build_levels(m.coords, m.coords, allv, 4 if dim == 2 else 8)
    Kl = K
    for l, P in enumerate(lv.prolong):
        Kl = hierarchy.galerkin(Kl, P, dim)
        X = lv.level_coords(l + 1)
        n = X.shape[0]
        modes = []
        for a in range(dim):
            u = np.zeros((n, dim)); u[:, a] = 1
            modes.append(u.ravel())
        for (a, b) in ([(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]):
            u = np.zeros((n, dim)); u[:, a] = -X[:, b]; u[:, b] = X[:, a]
            modes.append(u.ravel())
        R = np.array(modes).T
        assert np.abs(Kl @ R).max() < 1e-10 * abs(Kl).max() * max(1.0, np.abs(R).max())


def _sweep_order(o, l):
    """Unknown order of the coloured sweep: colours, colour blocks, cells,
    vertices, components."""
    d = o.d
    cell, block = o.cells[l], o.blocks[l]
    n = cell.size
    verts = np.lexsort((np.arange(n), cell, block, o.block_colors[l][block]))
    return np.array([v * d + a for v in verts for a in range(d)])


@pytest.mark.parametrize("dim", [2, 3])
def test_cells_and_coloring(dim):
    m = small2d(17, seed=1) if dim == 2 else small3d(9, seed=2)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(color_blocks="auto"))
    for l in range(o.L):
        S = o.S[l].tocoo()
        cell, col = o.cells[l], o.colors[l]
        sizes = np.bincount(cell)
        assert sizes.max() <= (1 if l == 0 else 2 ** dim)
        if l == 0:
            assert np.array_equal(cell, np.arange(cell.size))
        else:
            # cells are lattice blocks: all members share key // cell_side
            keys = o.levels.level_keys(l)
            side = 2 * int(tree.side_of(int(o.levels.regions[l - 1][0].max())))
            ck = keys // side
            for c in np.unique(cell):
                assert np.all(ck[cell == c] == ck[cell == c][0])
        # colour blocks: whole cells, lattice blocks of block_steps lattice steps,
        # coupled vertices of different blocks never share a colour
        block = o.blocks[l]
        for c in np.unique(cell):
            assert np.unique(block[cell == c]).size == 1
        offb = block[S.row] != block[S.col]
        assert np.all(col[S.row[offb]] == o.block_colors[l][block[S.row[offb]]])
        assert np.all(col[S.row[offb]] != col[S.col[offb]])
        if l > 0:
            h = int(tree.side_of(int(o.levels.regions[l - 1][0].max())))
            steps = o.block_steps[l]
            assert steps in (2, 4)
            bk = keys // (steps * h)
            for k in np.unique(block):
                assert np.all(bk[block == k] == bk[block == k][0])
            reach = hierarchy.coupling_reach(o.S[l], keys, h)
            if steps == 4:
                # blocks two apart along an axis are uncoupled: 2^d colours suffice
                assert dim == 3 and 2 < reach <= 4
                assert o.block_colors[l].max() + 1 <= 2 ** dim
            else:
                assert np.array_equal(block, cell)
                assert dim == 2 or not 2 < reach <= 4
        # the chosen colouring is the best of the greedy visiting orders
        nb = int(block.max()) + 1
        G = hierarchy.cell_graph(o.S[l], block, nb)
        canon = hierarchy.greedy_coloring_in_order(G, np.arange(nb))
        assert o.block_colors[l].max() <= canon.max()
    # coarse lattice levels of a near-uniform mesh reach 2^d colours
    assert o.cell_colors[o.L - 1].max() + 1 <= 2 ** dim
    # a 3D mesh of 2^k + 1 vertices per axis has a level 1 coupled 4 steps far:
    # colour blocks of 4 steps there
    if dim == 3:
        assert o.block_steps[1] == 4, o.block_steps


def _literal_gs(A, b, x, order):
    """Algorithm 1, one sweep, element by element, in the given unknown order."""
    x = x.copy()
    for i in order:
        sigma = 0.0
        for j in range(A.shape[0]):
            if j != i:
                sigma += A[i, j] * x[j]
        x[i] = (b[i] - sigma) / A[i, i]
    return x


@pytest.mark.parametrize("dim", [2, 3])
def test_gauss_seidel_orders(dim):
    m = _tiny(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    rng = np.random.default_rng(4)
    for l in range(min(o.L, 2)):
        A = o.A[l]
        Ad = A.toarray()
        n = A.shape[0]
        nv = n // dim
        b = rng.normal(size=n)
        x0 = rng.normal(size=n)
        order = list(_sweep_order(o, l))
        S = o.gs(l)
        assert np.allclose(S.forward(b, x0), _literal_gs(Ad, b, x0, order), rtol=1e-12, atol=1e-12)
        assert np.allclose(S.backward(b, x0), _literal_gs(Ad, b, x0, order[::-1]),
                           rtol=1e-12, atol=1e-12)
        # the paper's component-major order
        lex = [v * dim + a for a in range(dim) for v in range(nv)]
        G = LexGS(A, dim)
        assert np.allclose(G.forward(b, x0), _literal_gs(Ad, b, x0, lex), rtol=1e-12, atol=1e-12)
        assert np.allclose(G.backward(b, x0), _literal_gs(Ad, b, x0, lex[::-1]),
                           rtol=1e-12, atol=1e-12)
        # one forward sweep from zero = lower-triangular solve of the permuted matrix
        p = np.array(order)
        Ap = Ad[np.ix_(p, p)]
        y = np.linalg.solve(np.tril(Ap), b[p])
        z = np.empty(n); z[p] = y
        assert np.allclose(S.forward(b, np.zeros(n)), z, rtol=1e-12, atol=1e-12)


def test_gauss_seidel_order_with_color_blocks():
    """On a level swept by colour blocks the coloured sweep still equals the
    literal Algorithm 1 loop, in the order colours, blocks, cells, vertices,
    components (the blocks of a colour updated together, the cells of a block
    one after the other)."""
    m = small3d(9, seed=2)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(color_blocks="auto"))
    assert o.block_steps[1] == 4
    rng = np.random.default_rng(6)
    A = o.A[1]
    Ad = A.toarray()
    n = A.shape[0]
    b, x0 = rng.normal(size=n), rng.normal(size=n)
    order = list(_sweep_order(o, 1))
    S = o.gs(1)
    assert np.allclose(S.forward(b, x0), _literal_gs(Ad, b, x0, order), rtol=1e-12, atol=1e-12)
    assert np.allclose(S.backward(b, x0), _literal_gs(Ad, b, x0, order[::-1]), rtol=1e-12, atol=1e-12)
    # and it is a different order from the cells' own colouring
    o2 = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    assert not np.allclose(o2.gs(1).forward(b, x0), S.forward(b, x0))


def _closed_form_B(o, l, order_fn):
    """B_l = Mbar^{-1} + (I - M^{-T} A) P B_{l+1} P^T (I - A M^{-1}), M = lower
    triangle of A in the sweep order, Mbar^{-1} = M^{-1} + M^{-T} - M^{-T} A M^{-1}."""
    A = o.A[l].toarray()
    n = A.shape[0]
    if l == o.L:
        return np.linalg.inv(A)
    p = order_fn(l)
    Pm = np.zeros((n, n)); Pm[np.arange(n), p] = 1.0      # (Pm x)[k] = x[p[k]]
    M = Pm.T @ np.tril(Pm @ A @ Pm.T) @ Pm
    Mi = np.linalg.inv(M)
    Mbar = Mi + Mi.T - Mi.T @ A @ Mi
    Pb = hierarchy.block_prolongation(o.P[l], o.d).toarray()
    Bc = _closed_form_B(o, l + 1, order_fn)
    I = np.eye(n)
    return Mbar + (I - Mi.T @ A) @ Pb @ Bc @ Pb.T @ (I - A @ Mi)


@pytest.mark.parametrize("dim", [2, 3])
def test_vcycle_closed_form_spd(dim):
    m = _tiny(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    n = o.A[0].shape[0]
    B = dense_operator(lambda r: o.apply_precond(r), n)

    Bc = _closed_form_B(o, 0, lambda l: _sweep_order(o, l))
    assert np.abs(B - Bc).max() <= 1e-10 * np.abs(Bc).max()
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    # lexicographic smoother: same identities with the component-major order
    B2 = dense_operator(lambda r: o.apply_precond(r, smoother="lex"), n)

    def order_lex(l):
        nv = o.A[l].shape[0] // dim
        return np.array([v * dim + a for a in range(dim) for v in range(nv)])
    assert np.abs(B2 - _closed_form_B(o, 0, order_lex)).max() <= 1e-10 * np.abs(B2).max()
    ev = np.linalg.eigvals(B @ o.A[0].toarray()).real
    assert ev.min() > 0 and ev.max() <= 1.0 + 1e-10        # V(1,1) with exact coarse solve


def test_coarsest_is_fine_level_gives_exact_inverse():
    m = _tiny(2)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed,
               OracleOptions(coarsest_max_dofs=10 ** 6))
    assert o.L == 0
    x, info = o.solve(m.rhs[0], 1e-10)
    assert info["iterations"] == 1
    assert info["rel_res_true"] < 1e-12


def test_truncated_hierarchy_matches_prefix():
    m = small2d(13, seed=2)
    full = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    cut = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(coarsest_max_dofs=200))
    assert cut.L < full.L
    for l in range(cut.L + 1):
        assert abs(cut.A[l] - full.A[l]).max() == 0
    assert cut.A[cut.L].shape[0] <= 200 < cut.A[cut.L - 1].shape[0]


@pytest.mark.parametrize("dim", [2, 3])
def test_pcg_error_bound(dim):
    m = _tiny(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    A = o.A[0].toarray()
    b = o.to_free(m.rhs[0])
    xs = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    for rtol in (1e-4, 1e-8):
        x, info = o.solve(m.rhs[0], rtol)
        assert info["converged"]
        assert info["rel_res_true"] < rtol * 1.0001
        err = np.linalg.norm(o.to_free(x) - xs) / np.linalg.norm(xs)
        assert err <= kappa * rtol


def test_plain_cg_within_n_iterations():
    m = small2d(5, seed=1)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    n = o.A[0].shape[0]
    x, info = o.solve(m.rhs[0], 1e-10, precond="none")
    assert info["converged"] and info["iterations"] <= n


def test_pcg_zero_rhs_and_x0():
    m = small2d(7, seed=2)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    x, info = o.solve(np.zeros_like(m.rhs[0]), 1e-6)
    assert info["iterations"] == 0 and np.all(x == 0)
    x1, i1 = o.solve(m.rhs[0], 1e-3)
    x2, i2 = o.solve(m.rhs[0], 1e-8, x0=x1)
    assert i2["converged"] and i2["rel_res_true"] < 1e-8


def test_iterations_flat_under_refinement():
    """Theorem 3: kappa(B A) is bounded, so PCG iteration counts stay flat."""
    its = []
    for n in (17, 33, 65, 129):
        m = manufactured_mesh(n, seed=0)
        o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
        _, info = o.solve(m.rhs[0], 1e-6)
        its.append(info["iterations"])
    assert max(its) - min(its) <= 4, its
    assert max(its) <= 20, its


def test_fp32_vcycle_reaches_rtol():
    m = manufactured_mesh(33, seed=0)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    x64, i64 = o.solve(m.rhs[0], 1e-6)
    x32, i32 = o.solve(m.rhs[0], 1e-6, precision="fp32")
    assert i32["converged"] and i32["rel_res_true"] < 1e-6
    assert abs(i32["iterations"] - i64["iterations"]) <= 1
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-5


def test_jacobi_preconditioner():
    m = manufactured_mesh(17, seed=0)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    _, info = o.solve(m.rhs[0], 1e-6, precond="jacobi")
    assert info["converged"]


def test_no_boundary_conditions_is_degenerate():
    m = small2d(6, seed=1, fix="none")
    with pytest.raises(np.linalg.LinAlgError):
        Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)


def test_tree_over_free_vertices_option():
    m = small2d(9, seed=3)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(tree_vertices="free"))
    x, info = o.solve(m.rhs[0], 1e-6)
    assert info["converged"]


def test_sparse_helpers():
    S = sp.csr_matrix(np.array([[1, 1, 0], [1, 1, 1], [0, 1, 1]]))
    col = hierarchy.greedy_coloring(S)
    assert list(col) == [0, 1, 0]


def _closed_form_W(o, l, order_fn):
    """W-cycle: as the V-cycle closed form with the coarse operator of two visits,
    C = 2 B_{l+1} - B_{l+1} A_{l+1} B_{l+1} (x0 + B (b - A x0) applied twice from 0);
    one visit of the coarsest level (exact solve)."""
    A = o.A[l].toarray()
    n = A.shape[0]
    if l == o.L:
        return np.linalg.inv(A)
    p = order_fn(l)
    Pm = np.zeros((n, n)); Pm[np.arange(n), p] = 1.0
    M = Pm.T @ np.tril(Pm @ A @ Pm.T) @ Pm
    Mi = np.linalg.inv(M)
    Mbar = Mi + Mi.T - Mi.T @ A @ Mi
    Pb = hierarchy.block_prolongation(o.P[l], o.d).toarray()
    B1 = _closed_form_W(o, l + 1, order_fn)
    if l + 1 < o.L:
        A1 = o.A[l + 1].toarray()
        C = 2.0 * B1 - B1 @ A1 @ B1
    else:
        C = B1
    I = np.eye(n)
    return Mbar + (I - Mi.T @ A) @ Pb @ C @ Pb.T @ (I - A @ Mi)


@pytest.mark.parametrize("dim", [2, 3])
def test_w_cycle_closed_form_spd(dim):
    m = small2d(9, seed=1) if dim == 2 else small3d(5, seed=2)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    assert o.L >= 3                      # the W-cycle differs from the V-cycle
    n = o.A[0].shape[0]
    B = dense_operator(lambda r: o.vcycle(cycle="W").apply(r), n)
    Bc = _closed_form_W(o, 0, lambda l: _sweep_order(o, l))
    assert np.abs(B - Bc).max() <= 1e-10 * np.abs(Bc).max()
    assert np.abs(B - B.T).max() <= 1e-11 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    BV = dense_operator(lambda r: o.vcycle(cycle="V").apply(r), n)
    assert np.abs(B - BV).max() > 1e-6 * np.abs(BV).max()


def test_w_cycle_equals_v_cycle_on_two_levels():
    m = small2d(13, seed=3)          # levels of 242, 162, 50, ... DOFs
    full = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed,
               OracleOptions(coarsest_max_dofs=full.A[1].shape[0]))
    assert o.L == 1
    r = np.random.default_rng(0).normal(size=o.A[0].shape[0])
    assert np.array_equal(o.vcycle(cycle="W").apply(r), o.vcycle(cycle="V").apply(r))


@pytest.mark.parametrize("dim", [2, 3])
def test_additive_two_level_closed_form_spd(dim):
    """B = Mbar_0^{-1} + P_0 B_1 P_0^T with B_1 the V-cycle of levels 1..L."""
    m = _tiny(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    n = o.A[0].shape[0]
    B = dense_operator(lambda r: o.vcycle(cycle="additive").apply(r), n)
    A = o.A[0].toarray()
    p = _sweep_order(o, 0)
    Pm = np.zeros((n, n)); Pm[np.arange(n), p] = 1.0
    Mi = np.linalg.inv(Pm.T @ np.tril(Pm @ A @ Pm.T) @ Pm)
    Mbar = Mi + Mi.T - Mi.T @ A @ Mi
    Pb = hierarchy.block_prolongation(o.P[0], o.d).toarray()
    Bc = Mbar + Pb @ _closed_form_B(o, 1, lambda l: _sweep_order(o, l)) @ Pb.T
    assert np.abs(B - Bc).max() <= 1e-10 * np.abs(Bc).max()
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0


def test_cycle_variants_converge():
    m = small2d(33, seed=4)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    its = {}
    for c in ("V", "W", "additive"):
        o2 = Oracle.__new__(Oracle)
        o2.__dict__.update(o.__dict__)
        o2._vcycles = {}
        o2.opts = OracleOptions(cycle=c)
        x, info = o2.solve(m.rhs[0], 1e-8)
        assert info["rel_res_true"] < 1e-8
        its[c] = info["iterations"]
    print(its)
    assert its["W"] <= its["V"] + 1 and its["additive"] >= its["V"] - 1


@pytest.mark.parametrize("dim", [2, 3])
def test_block_jacobi_smoother(dim):
    """Damped vertex-block Jacobi (Section 4's Jacobi option for S_h): the step is
    x + omega D^{-1} (b - A x); the power-iteration estimate is within 10% below
    the true lambda_max(D^{-1} A), so omega * lambda_max < 2; the V-cycle with it
    is symmetric positive definite and PCG converges."""
    from oracle.smoother import BlockJacobi
    m = _tiny(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    A = o.A[0]
    Ad = A.toarray()
    n = Ad.shape[0]
    D = np.zeros_like(Ad)
    for k in range(n // dim):
        sl = slice(k * dim, (k + 1) * dim)
        D[sl, sl] = Ad[sl, sl]
    lam_true = np.linalg.eigvals(np.linalg.solve(D, Ad)).real.max()
    J = BlockJacobi(A, dim)
    assert 0.9 * lam_true <= J.lam <= lam_true * (1 + 1e-12)
    assert J.omega * lam_true < 2.0
    rng = np.random.default_rng(1)
    b, x = rng.normal(size=n), rng.normal(size=n)
    ref = x + J.omega * np.linalg.solve(D, b - Ad @ x)
    assert np.allclose(J.forward(b, x), ref, rtol=1e-12, atol=1e-12)
    B = dense_operator(lambda r: o.apply_precond(r, smoother="jacobi"), n)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    xs, info = o.solve(m.rhs[0], 1e-8, smoother="jacobi")
    assert info["rel_res_true"] < 1e-8
