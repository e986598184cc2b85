"""Pins of partially constrained vertices (homogeneous Dirichlet conditions on
some components of a vertex; Section 2, boundary conditions of the system).

The oracle keeps such a vertex's block with an identity row and column for each
fixed component and zero prolongation rows for it; a coarse component all of
whose interpolating fine vertices have it fixed is constrained in turn. That
is exactly eliminating the fixed components. (Zeroed rows can leave dependent
prolongation columns, so a coarse operator may be only semi-definite, in both
forms alike; Gauss-Seidel needs only its positive diagonal.) The pins build the eliminated
form independently (rows and columns deleted, its own Galerkin products, a
literal Gauss-Seidel loop in the same unknown order, a dense coarsest solve)
and require:
  * identical level operators on the unconstrained DOFs, and unit rows and
    columns at the constrained ones;
  * identical z = B r on the unconstrained DOFs, and z = 0 at the constrained;
  * the PCG solution of a roller (symmetry-plane) problem equal to a dense
    direct solve of the eliminated system.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleOptions
from oracle.hierarchy import block_prolongation
from workloads import small2d, small3d

MESHES = {
    "2d_symmetry": lambda: small2d(9, seed=1, fix="symmetry"),
    "3d_symmetry": lambda: small3d(5, seed=2, fix="symmetry"),
    "3d_clamp_rollers": lambda: small3d(7, seed=3, fix="roller_x1"),
}


def _eliminated(o, m):
    """Level operators, prolongations and kept DOFs of the eliminated form."""
    d = o.d
    fixed = np.asarray(m.fixed).astype(bool)
    dofs = np.array([v * d + a for v in o.free for a in range(d) if not fixed[v, a]])
    A = [o.K[dofs][:, dofs].toarray()]
    keep = [np.flatnonzero(~fixed[o.free].ravel())]
    P = []
    for l in range(o.L):
        Pb = block_prolongation(o.P[l], d).toarray()[keep[l]]
        cols = np.flatnonzero(np.abs(Pb).sum(axis=0) > 0)
        P.append(Pb[:, cols])
        keep.append(cols)
        A.append(P[l].T @ A[l] @ P[l])
    return A, P, keep


def _order(o, l, keep):
    """The oracle's unknown order on level l restricted to the kept DOFs, as
    positions in the kept list."""
    d = o.d
    n = o.A[l].shape[0] // d
    if l == o.L:
        return None
    verts = np.lexsort((np.arange(n), o.cells[l], o.blocks[l], o.colors[l]))
    order = np.array([v * d + a for v in verts for a in range(d)])
    pos = np.full(n * d, -1)
    pos[keep] = np.arange(keep.size)
    return pos[order][pos[order] >= 0]


def _gs(A, b, x, order):
    x = x.copy()
    for i in order:
        x[i] = (b[i] - A[i] @ x + A[i, i] * x[i]) / A[i, i]
    return x


def _vcycle(o, A, P, keep, l, b):
    if l == o.L:
        return np.linalg.solve(A[l], b)
    order = _order(o, l, keep[l])
    x = _gs(A[l], b, np.zeros_like(b), order)
    r = b - A[l] @ x
    e = _vcycle(o, A, P, keep, l + 1, P[l].T @ r)
    x = x + P[l] @ e
    return _gs(A[l], b, x, order[::-1])


@pytest.mark.parametrize("name", list(MESHES))
def test_identity_rows_equal_elimination_level_by_level(name):
    m = MESHES[name]()
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    fixed = np.asarray(m.fixed).astype(bool)
    # DOFs: every vertex with a free component keeps its block
    assert o.A[0].shape[0] == m.dim * np.count_nonzero(~fixed.all(axis=1))
    assert np.array_equal(o.cmask[0], fixed[o.free].ravel())
    A, P, keep = _eliminated(o, m)
    for l in range(o.L + 1):
        Al = o.A[l].toarray()
        cm = o.cmask[l]
        assert np.array_equal(np.flatnonzero(~cm), keep[l]), l
        # unit rows and columns at constrained DOFs
        assert np.array_equal(Al[cm], np.eye(Al.shape[0])[cm]), l
        assert np.array_equal(Al[:, cm], np.eye(Al.shape[0])[:, cm]), l
        # the rest is the eliminated operator
        Ak = Al[np.ix_(keep[l], keep[l])]
        assert np.abs(Ak - A[l]).max() <= 1e-13 * np.abs(A[l]).max(), l
        # symmetric positive semi-definite with a positive diagonal (zeroed
        # prolongation rows can leave dependent columns: the eliminated form
        # has the same operator); the fine and coarsest levels definite
        ev = np.linalg.eigvalsh(Al)
        assert np.all(np.diag(Al) > 0)
        assert ev[0] >= -1e-13 * ev[-1], l
        if l in (0, o.L):
            assert ev[0] > 0, l


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("cycle", ["V", "W"])
def test_identity_rows_equal_elimination_in_the_cycle(name, cycle):
    m = MESHES[name]()
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(cycle=cycle))
    A, P, keep = _eliminated(o, m)
    rng = np.random.default_rng(5)
    r = rng.normal(size=o.A[0].shape[0])
    r[o.cmask[0]] = 0.0
    z = o.apply_precond(r)
    assert np.all(z[o.cmask[0]] == 0.0)
    if cycle == "V":
        ze = _vcycle(o, A, P, keep, 0, r[keep[0]])
        assert np.abs(z[keep[0]] - ze).max() <= 1e-12 * np.abs(ze).max()
    else:
        # the W-cycle's extra coarse visits keep the constrained DOFs at zero too
        zv = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed).apply_precond(r)
        assert np.linalg.norm(z - zv) > 0


@pytest.mark.parametrize("name", list(MESHES))
def test_roller_solve_matches_dense_solve(name):
    m = MESHES[name]()
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    A, _, keep = _eliminated(o, m)
    F = o.to_free(m.rhs[0])
    assert np.all(F[o.cmask[0]] == 0.0)
    xe = np.linalg.solve(A[0], F[keep[0]])
    x, info = o.solve(m.rhs[0], 1e-12)
    assert info["converged"]
    xf = o.to_free(x)
    kappa = np.linalg.cond(A[0])
    assert np.linalg.norm(xf[keep[0]] - xe) <= kappa * 1e-12 * np.linalg.norm(xe)
    assert np.all(x[np.asarray(m.fixed).astype(bool)] == 0.0)
    # the Jacobi-smoothed cycle and the FP32 cycle keep the same solution
    for kw in (dict(smoother="jacobi"), dict(precision="fp32")):
        x2, i2 = o.solve(m.rhs[0], 1e-10, **kw)
        assert i2["converged"]
        assert np.linalg.norm(o.to_free(x2)[keep[0]] - xe) <= 1e-7 * np.linalg.norm(xe)


def test_coarse_constraints_are_exercised():
    """The meshes above reach the propagation rule: coarse components
    constrained because every interpolating fine vertex has them fixed."""
    n = 0
    for name in ("2d_symmetry", "3d_symmetry"):
        m = MESHES[name]()
        o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
        n_coarse = sum(int(c.sum()) for c in o.cmask[1:])
        assert n_coarse > 0, name
        n += n_coarse
    assert n > 0
