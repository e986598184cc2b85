"""Pins of the oracle's P1 elasticity assembly (Section 2 of the paper).

Each test checks the oracle against something other than itself: the kernel of
the unconstrained operator (rigid-body modes), the patch test,
symmetry up to rounding, positive definiteness after Dirichlet elimination, the paper's 2x2
operator-block form, and the O(h^2) convergence of a manufactured solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve

from oracle import fem
from workloads import grid2d, grid3d, manufactured_2d, manufactured_mesh


def _rigid_modes(coords):
    d = coords.shape[1]
    n = coords.shape[0]
    modes = []
    for a in range(d):
        u = np.zeros((n, d)); u[:, a] = 1.0
        modes.append(u.ravel())
    pairs = [(0, 1)] if d == 2 else [(0, 1), (0, 2), (1, 2)]
    for (a, b) in pairs:                      # infinitesimal rotation in the (a, b) plane
        u = np.zeros((n, d)); u[:, a] = -coords[:, b]; u[:, b] = coords[:, a]
        modes.append(u.ravel())
    return np.array(modes).T


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_body_kernel(dim):
    """The unconstrained stiffness matrix has exactly the rigid-body modes as kernel."""
    if dim == 2:
        coords, el, _ = grid2d(6, seed=11)
    else:
        coords, el, _ = grid3d(4, seed=12)
    K = fem.assemble(coords, el, 1.0, 0.3)
    R = _rigid_modes(coords)
    scale = abs(K).max()
    assert np.abs(K @ R).max() < 1e-12 * scale
    ev = np.linalg.eigvalsh(K.toarray())
    nker = 3 if dim == 2 else 6
    assert np.all(np.abs(ev[:nker]) < 1e-10 * ev[-1])
    assert ev[nker] > 1e-6 * ev[-1]


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test(dim):
    """A linear displacement field is in equilibrium at every interior vertex."""
    if dim == 2:
        coords, el, bnd = grid2d(7, seed=3)
    else:
        coords, el, bnd = grid3d(5, seed=4)
    rng = np.random.default_rng(0)
    a = rng.normal(size=dim)
    B = rng.normal(size=(dim, dim))
    u = (a[None, :] + coords @ B.T).ravel()
    K = fem.assemble(coords, el, 1.0, 0.3)
    f = (K @ u).reshape(-1, dim)
    assert np.abs(f[~bnd]).max() < 1e-12 * abs(K).max() * np.abs(u).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_and_spd(dim):
    if dim == 2:
        coords, el, bnd = grid2d(6, seed=5)
    else:
        coords, el, bnd = grid3d(4, seed=6)
    rng = np.random.default_rng(1)
    E = rng.uniform(1, 100, el.shape[0])
    nu = rng.uniform(0.1, 0.49, el.shape[0])
    K = fem.assemble(coords, el, E, nu)
    assert abs(K - K.T).max() <= 4 * np.finfo(float).eps * abs(K).max()
    fixed = np.zeros((coords.shape[0], dim), np.uint8)
    fixed[bnd] = 1
    free = fem.free_vertices(fixed)
    A = fem.restrict_free(K, free, dim).toarray()
    assert np.linalg.eigvalsh(A)[0] > 0


def test_block_form_of_the_paper():
    """The vertex-major matrix equals the paper's [[lam A11 + 2mu A11 + mu A22, ...]] form."""
    coords, el, _ = grid2d(7, seed=8)
    rng = np.random.default_rng(2)
    E = rng.uniform(1, 10, el.shape[0])
    nu = rng.uniform(0.2, 0.45, el.shape[0])
    K = fem.assemble(coords, el, E, nu)
    Kb = fem.assemble_block_form_2d(coords, el, E, nu)
    perm = fem.component_major_perm(coords.shape[0], 2)
    Kcm = K[perm][:, perm]
    assert abs(Kcm - Kb).max() < 1e-13 * abs(Kb).max()


def test_lame_constants():
    mu, lam = fem.lame(1.0, 0.3)
    assert mu == pytest.approx(1 / 2.6)
    assert lam == pytest.approx(0.3 / (1.3 * 0.4))
    mu, lam = fem.lame(1.0, 0.49)
    assert lam == pytest.approx(16.44295302, rel=1e-8)


def test_manufactured_solution_converges_at_second_order():
    """Discrete L2 nodal error of the manufactured solution decays like h^2."""
    u_exact, _ = manufactured_2d(1.0, 0.3)
    errs = []
    ns = [17, 33, 65]
    for n in ns:
        m = manufactured_mesh(n, seed=0)
        K = fem.assemble(m.coords, m.elems, m.E, m.nu)
        free = fem.free_vertices(m.fixed)
        A = fem.restrict_free(K, free, 2)
        b = m.rhs[0][free].ravel()
        x = spsolve(A.tocsc(), b).reshape(-1, 2)
        ue = u_exact(m.coords[free, 0], m.coords[free, 1])
        h = 1.0 / (n - 1)
        errs.append(np.sqrt(h * h * np.sum((x - ue) ** 2)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > 1.8, rates
    assert errs[-1] < 1e-3


def test_partially_fixed_vertices_keep_their_block():
    """Only fully fixed vertices are eliminated; a fixed component of another
    vertex gets an identity row and column (tests/test_oracle_constraints.py
    pins that this equals eliminating it)."""
    fixed = np.zeros((4, 2), np.uint8)
    fixed[0, 0] = 1
    fixed[1] = 1
    free = fem.free_vertices(fixed)
    assert np.array_equal(free, [0, 2, 3])
    assert np.array_equal(fem.constrained_dofs(fixed, free), [1, 0, 0, 0, 0, 0])


def test_fine_pattern_matches_matrix():
    coords, el, bnd = grid3d(4, seed=2)
    fixed = np.zeros((coords.shape[0], 3), np.uint8)
    fixed[coords[:, 0] == 0] = 1
    free = fem.free_vertices(fixed)
    K = fem.assemble(coords, el, 1.0, 0.3)
    A = fem.restrict_free(K, free, 3)
    S = fem.fine_pattern(el, free, coords.shape[0])
    Ablk = abs(A).tocsr()
    # block (i, j) is nonzero only where vertices share an element
    Bn = sp.csr_matrix((np.ones(Ablk.nnz), Ablk.indices, Ablk.indptr), shape=A.shape)
    V = sp.kron(S, np.ones((3, 3)), format="csr")
    assert (Bn > 0).multiply(V == 0).nnz == 0
