"""Seeded synthetic P1 meshes and load vectors for the V-ASMG-PCG workloads.

The paper's eight engineering meshes (its Section 5) are not available, so
these structured-then-jittered (or graded) meshes on the unit square/cube
stand in for them, with the paper's value ranges for E and nu (Section 5,
Examples 4.1-4.8) and its P1 element type.

Conventions (shared by every consumer):
  * vertex index = i + n_x*(j + n_y*k), x fastest;
  * coordinates on [0,1]^d; jitter is drawn with numpy's default_rng(seed) as
    uniform(-0.2h, 0.2h) for ALL vertices in index order, then zeroed on
    boundary vertices;
  * triangles: each square is split along its lower-left -> upper-right
    diagonal into (v00,v10,v11) and (v00,v11,v01), counter-clockwise;
  * tetrahedra: each cube is split into the 6 Kuhn tetrahedra around its
    (0,0,0)->(1,1,1) diagonal, reoriented to positive volume;
  * the load vector F[v, a] = sum over elements e of int_e f_a phi_v is an
    input to the solver (the paper's F, Section 2); it is computed here by
    quadrature (edge-midpoint rule on triangles, the 4-point degree-2 rule on
    tetrahedra, exact |e|/(d+1) for constant f).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

JITTER = 0.2


@dataclass
class Mesh:
    name: str
    dim: int
    coords: np.ndarray            # [Nv, d] float64
    elems: np.ndarray             # [Ne, d+1] int32, positively oriented
    E: np.ndarray                 # [Ne] float64 Young's modulus per element
    nu: np.ndarray                # [Ne] float64 Poisson ratio per element
    fixed: np.ndarray             # [Nv, d] uint8, 1 = homogeneous Dirichlet DOF
    rhs: list = field(default_factory=list)   # list of [Nv, d] float64 load vectors

    @property
    def n_vertices(self) -> int:
        return self.coords.shape[0]

    @property
    def n_free_vertices(self) -> int:
        return int(np.count_nonzero(~self.fixed.any(axis=1)))

    @property
    def n_dofs(self) -> int:
        return self.dim * self.n_free_vertices


# --------------------------------------------------------------------------
# vertex grids
# --------------------------------------------------------------------------

def _axis(n: int, graded: bool) -> np.ndarray:
    t = np.arange(n, dtype=np.float64) / (n - 1)
    return t * t if graded else t


def _jitter(coords: np.ndarray, boundary: np.ndarray, h: float, seed) -> np.ndarray:
    rng = np.random.default_rng(seed)
    J = rng.uniform(-JITTER * h, JITTER * h, size=coords.shape)
    J[boundary] = 0.0
    return coords + J


def grid2d(n: int, seed=None, graded: bool = False):
    """n x n vertices on [0,1]^2; returns (coords, tris, boundary_mask)."""
    ax = _axis(n, graded)
    X, Y = np.meshgrid(ax, ax, indexing="xy")          # Y[j, i], X[j, i]
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii = ii.ravel(); jj = jj.ravel()
    boundary = (ii == 0) | (jj == 0) | (ii == n - 1) | (jj == n - 1)
    if seed is not None:
        coords = _jitter(coords, boundary, 1.0 / (n - 1), seed)
    ci, cj = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    ci = ci.ravel(); cj = cj.ravel()
    v00 = ci + n * cj
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tris = np.empty((2 * t1.shape[0], 3), dtype=np.int32)
    tris[0::2] = t1
    tris[1::2] = t2
    return coords, tris, boundary


_KUHN = [  # offsets (dx,dy,dz) of the 4 vertices of the 6 Kuhn tetrahedra
    ((0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1)),
    ((0, 0, 0), (1, 0, 0), (1, 0, 1), (1, 1, 1)),
    ((0, 0, 0), (0, 1, 0), (1, 1, 0), (1, 1, 1)),
    ((0, 0, 0), (0, 1, 0), (0, 1, 1), (1, 1, 1)),
    ((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1)),
    ((0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1)),
]


def grid3d(n: int, seed=None):
    """n^3 vertices on [0,1]^3; returns (coords, tets, boundary_mask)."""
    return _grid3d(n, n, n, 1.0 / (n - 1), _axis(n, False), seed)


def grid3d_box(nx: int, ny: int, nz: int, h: float, seed=None):
    """nx x ny x nz vertices with spacing h on [0,(nx-1)h] x [0,(ny-1)h] x
    [0,(nz-1)h]; returns (coords, tets, boundary_mask)."""
    return _grid3d(nx, ny, nz, h, None, seed)


def _grid3d(nx, ny, nz, h, axis, seed):
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ii = ii.ravel(); jj = jj.ravel(); kk = kk.ravel()
    if axis is not None:
        coords = np.stack([axis[ii], axis[jj], axis[kk]], axis=1)
    else:
        coords = np.stack([ii * h, jj * h, kk * h], axis=1).astype(np.float64)
    boundary = ((ii == 0) | (jj == 0) | (kk == 0)
                | (ii == nx - 1) | (jj == ny - 1) | (kk == nz - 1))
    if seed is not None:
        coords = _jitter(coords, boundary, h, seed)
    ck, cj, ci = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    base = (ci + nx * (cj + ny * ck)).ravel()
    tets = []
    for offs in _KUHN:
        idx = [base + dx + nx * (dy + ny * dz) for (dx, dy, dz) in offs]
        # orientation of this tet type on the reference cube
        P = np.array(offs, dtype=np.float64)
        if np.linalg.det(P[1:] - P[0]) < 0:
            idx[2], idx[3] = idx[3], idx[2]
        tets.append(np.stack(idx, axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return coords, tets, boundary


def signed_measure(coords: np.ndarray, elems: np.ndarray) -> np.ndarray:
    """det of the edge matrix of each element (2x area / 6x volume)."""
    X = coords[elems[:, 1:]] - coords[elems[:, :1]]
    return np.linalg.det(X)


# --------------------------------------------------------------------------
# load vectors (inputs to the solver)
# --------------------------------------------------------------------------

def _measure(coords, elems):
    d = elems.shape[1] - 1
    fact = 2.0 if d == 2 else 6.0
    return np.abs(signed_measure(coords, elems)) / fact


def load_constant(coords, elems, f) -> np.ndarray:
    """F for a constant body force f (exact: |e|/(d+1) per vertex)."""
    d = coords.shape[1]
    vol = _measure(coords, elems)
    F = np.zeros((coords.shape[0], d))
    share = vol / (d + 1)
    for a in range(d + 1):
        np.add.at(F, elems[:, a], share[:, None] * np.asarray(f, dtype=np.float64)[None, :])
    return F


def load_function_tri(coords, elems, fun) -> np.ndarray:
    """F on triangles by the edge-midpoint rule (weights |e|/3, exact to degree 2).

    fun(x, y) -> [n, 2] values. At the midpoint of edge (a,b) phi_a = phi_b = 1/2
    and the third basis function vanishes.
    """
    vol = _measure(coords, elems)
    F = np.zeros((coords.shape[0], 2))
    for (a, b) in ((0, 1), (1, 2), (2, 0)):
        m = 0.5 * (coords[elems[:, a]] + coords[elems[:, b]])
        fv = fun(m[:, 0], m[:, 1])
        contrib = (vol / 3.0)[:, None] * fv * 0.5
        np.add.at(F, elems[:, a], contrib)
        np.add.at(F, elems[:, b], contrib)
    return F


_TET_A = 0.5854101966249685
_TET_B = 0.1381966011250105


def load_function_tet(coords, elems, fun) -> np.ndarray:
    """F on tetrahedra by the symmetric 4-point degree-2 rule (weights |e|/4)."""
    vol = _measure(coords, elems)
    F = np.zeros((coords.shape[0], 3))
    X = coords[elems]                        # [Ne, 4, 3]
    for q in range(4):
        lam = np.full(4, _TET_B); lam[q] = _TET_A
        p = np.einsum("k,ekd->ed", lam, X)
        fv = fun(p[:, 0], p[:, 1], p[:, 2])   # [Ne, 3]
        for a in range(4):
            np.add.at(F, elems[:, a], (vol / 4.0 * lam[a])[:, None] * fv)
    return F


def lame(E, nu):
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def manufactured_2d(E: float = 1.0, nu: float = 0.3):
    """u = (sin(pi x) sin(pi y), x(1-x)y(1-y)) and f = -div sigma(u) (plane strain)."""
    mu, lam = lame(E, nu)
    pi = np.pi

    def u(x, y):
        return np.stack([np.sin(pi * x) * np.sin(pi * y), x * (1 - x) * y * (1 - y)], axis=-1)

    def f(x, y):
        f1 = (lam + 3 * mu) * pi ** 2 * np.sin(pi * x) * np.sin(pi * y) \
            - (lam + mu) * (1 - 2 * x) * (1 - 2 * y)
        f2 = 2 * mu * y * (1 - y) + (2 * lam + 4 * mu) * x * (1 - x) \
            - (lam + mu) * pi ** 2 * np.cos(pi * x) * np.cos(pi * y)
        return np.stack([f1, f2], axis=-1)

    return u, f


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def small2d(n: int = 9, seed=0, E: float = 1.0, nu: float = 0.3, fix: str = "boundary",
            f=(0.0, -1.0), graded: bool = False) -> Mesh:
    coords, tris, bnd = grid2d(n, seed, graded)
    fixed = np.zeros((coords.shape[0], 2), dtype=np.uint8)
    if fix == "boundary":
        fixed[bnd] = 1
    elif fix == "x0":
        fixed[np.isclose(coords[:, 0], 0.0)] = 1
    elif fix == "symmetry":
        # rollers: u_x = 0 on x = 0, u_y = 0 on y = 0 (the corner is fully fixed)
        fixed[coords[:, 0] == 0.0, 0] = 1
        fixed[coords[:, 1] == 0.0, 1] = 1
    elif fix == "none":
        pass
    else:
        raise ValueError(fix)
    ne = tris.shape[0]
    F = load_constant(coords, tris, f)
    return Mesh(f"small2d_n{n}", 2, coords, tris, np.full(ne, E), np.full(ne, nu), fixed, [F])


def small3d(n: int = 5, seed=1, E: float = 1.0, nu: float = 0.3, fix: str = "x0",
            f=(0.0, 0.0, -1.0)) -> Mesh:
    coords, tets, bnd = grid3d(n, seed)
    fixed = np.zeros((coords.shape[0], 3), dtype=np.uint8)
    if fix == "boundary":
        fixed[bnd] = 1
    elif fix == "x0":
        fixed[coords[:, 0] == 0.0] = 1
    elif fix == "symmetry":
        # rollers on the three coordinate planes: u_a = 0 on x_a = 0 (edges fix
        # two components, the corner all three)
        for a in range(3):
            fixed[coords[:, a] == 0.0, a] = 1
    elif fix == "roller_x1":
        # clamped at x = 1, rollers u_y = 0 on y = 0 and u_z = 0 on z = 0
        fixed[coords[:, 0] == 1.0] = 1
        fixed[coords[:, 1] == 0.0, 1] = 1
        fixed[coords[:, 2] == 0.0, 2] = 1
    elif fix == "none":
        pass
    else:
        raise ValueError(fix)
    ne = tets.shape[0]
    F = load_constant(coords, tets, f)
    return Mesh(f"small3d_n{n}", 3, coords, tets, np.full(ne, E), np.full(ne, nu), fixed, [F])


def box3d(nx: int, ny: int, nz: int, seed=1, E: float = 1.0, nu: float = 0.3,
          f=(0.0, 0.0, -1.0)) -> Mesh:
    """3D box of nx x ny x nz vertices, spacing h = 1/(nz-1) (so z spans [0,1]),
    jittered by +-0.2h (seed), Kuhn tetrahedra, clamped at x=0, constant body
    force f."""
    h = 1.0 / (nz - 1)
    coords, tets, _ = grid3d_box(nx, ny, nz, h, seed)
    fixed = np.zeros((coords.shape[0], 3), dtype=np.uint8)
    fixed[coords[:, 0] == 0.0] = 1
    ne = tets.shape[0]
    F = load_constant(coords, tets, f)
    return Mesh(f"box3d_{nx}x{ny}x{nz}", 3, coords, tets, np.full(ne, E), np.full(ne, nu), fixed,
                [F])


def manufactured_mesh(n: int, seed=0, E: float = 1.0, nu: float = 0.3) -> Mesh:
    """2D plane strain, n x n jittered grid, all boundary fixed, manufactured f."""
    coords, tris, bnd = grid2d(n, seed)
    fixed = np.zeros((coords.shape[0], 2), dtype=np.uint8)
    fixed[bnd] = 1
    _, f = manufactured_2d(E, nu)
    F = load_function_tri(coords, tris, f)
    ne = tris.shape[0]
    return Mesh(f"manufactured_n{n}", 2, coords, tris, np.full(ne, E), np.full(ne, nu), fixed, [F])


def cfg1() -> Mesh:
    """2D plane strain, 33x33 jittered grid (seed 0), manufactured solution, 1,922 DOFs."""
    m = manufactured_mesh(33, seed=0)
    m.name = "cfg1_2d_33x33_manufactured"
    return m


def cfg2() -> Mesh:
    """3D, 65^3 jittered grid (seed 1), Kuhn tets, clamped at x=0, f=(0,0,-1); 811,200 DOFs."""
    m = small3d(65, seed=1, fix="x0")
    m.name = "cfg2_3d_65cubed_clamped"
    return m


def cfg3() -> Mesh:
    """2D nu=0.49, 1025^2 graded grid (x->x^2, y->y^2), E in {1,100} on a seeded 8x8
    checkerboard (seed 2), all boundary fixed, f=(0,-1); 2,093,058 DOFs."""
    coords, tris, bnd = grid2d(1025, None, graded=True)
    fixed = np.zeros((coords.shape[0], 2), dtype=np.uint8)
    fixed[bnd] = 1
    cen = coords[tris].mean(axis=1)
    bx = np.minimum((cen[:, 0] * 8).astype(np.int64), 7)
    by = np.minimum((cen[:, 1] * 8).astype(np.int64), 7)
    table = np.random.default_rng(2).random(64)
    E = np.where(table[bx + 8 * by] < 0.5, 100.0, 1.0)
    nu = np.full(tris.shape[0], 0.49)
    F = load_constant(coords, tris, (0.0, -1.0))
    return Mesh("cfg3_2d_1025sq_graded_nu049", 2, coords, tris, E, nu, fixed, [F])


def _fourier_modes(r: int, seed: int):
    """Modes of load case r: per component, 8 (k in {1..4}^3, c ~ N(0,1)) pairs."""
    rng = np.random.default_rng([seed, r])
    modes = []
    for a in range(3):
        ma = []
        for _ in range(8):
            k = rng.integers(1, 5, size=3)
            c = rng.normal()
            ma.append((k, c))
        modes.append(ma)
    return modes


def fourier_body_force(r: int, seed: int = 3):
    """Column r of the smooth random body forces (8 Fourier modes per component):
    f_a = sum_m c_m sin(pi k1 x) sin(pi k2 y) sin(pi k3 z)."""
    modes = _fourier_modes(r, seed)

    def f(x, y, z):
        out = np.zeros((x.shape[0], 3))
        for a in range(3):
            for (k, c) in modes[a]:
                out[:, a] += c * np.sin(np.pi * k[0] * x) * np.sin(np.pi * k[1] * y) \
                    * np.sin(np.pi * k[2] * z)
        return out
    return f


def load_fourier_tet(coords, elems, n_rhs: int, seed: int = 3, chunk: int = 1 << 18):
    """The first n_rhs Fourier body-force load cases at once, by the same 4-point
    degree-2 rule as load_function_tet (equal values up to summation order).

    At each quadrature point the 64 products sin(pi k1 x) sin(pi k2 y)
    sin(pi k3 z), k in {1..4}^3, times a [64, 3 n_rhs] coefficient matrix give
    every load case's components; element slot s receives |e|/4 (B sum_q f_q +
    (A - B) f_s), accumulated into the vertex rows by a sparse incidence product
    that adds into the output in place. Elements go in chunks through work
    arrays allocated once (first-touch page faults, not arithmetic, dominate
    fresh large temporaries)."""
    import scipy.sparse as sp
    from scipy.sparse import _sparsetools
    nv, ne = coords.shape[0], elems.shape[0]
    R3 = 3 * n_rhs
    Cm = np.zeros((64, R3))
    for r in range(n_rhs):
        for a, ma in enumerate(_fourier_modes(r, seed)):
            for (k, c) in ma:
                Cm[(k[0] - 1) * 16 + (k[1] - 1) * 4 + (k[2] - 1), 3 * r + a] += c
    kk = np.pi * np.arange(1, 5)[:, None]
    m = min(chunk, ne)
    t = np.empty((3, 4, m))
    t01 = np.empty((4, 4, m))
    P = np.empty((4, 4, 4, m))
    fq = np.empty((4, m, R3))
    fsum = np.empty((m, R3))
    share = np.empty((m, R3))
    F = np.zeros((nv, R3))
    for e0 in range(0, ne, chunk):
        el = elems[e0:e0 + chunk]
        n = el.shape[0]
        vol4 = _measure(coords, el) / 4.0
        X = coords[el]
        for q in range(4):
            lam = np.full(4, _TET_B); lam[q] = _TET_A
            pq = np.einsum("k,ekd->de", lam, X)
            for d in range(3):
                np.multiply(kk, pq[d][None, :], out=t[d, :, :n])
                np.sin(t[d, :, :n], out=t[d, :, :n])
            np.multiply(t[0, :, None, :n], t[1, None, :, :n], out=t01[:, :, :n])
            np.multiply(t01[:, :, None, :n], t[2, None, None, :, :n], out=P[:, :, :, :n])
            Pv = P.reshape(64, m)[:, :n] if n == m else np.ascontiguousarray(P[:, :, :, :n]).reshape(64, n)
            np.matmul(Pv.T, Cm, out=fq[q, :n])
        np.add(fq[0, :n], fq[1, :n], out=fsum[:n])
        np.add(fsum[:n], fq[2, :n], out=fsum[:n])
        np.add(fsum[:n], fq[3, :n], out=fsum[:n])
        fsum[:n] *= _TET_B
        cols = np.arange(n)
        for sl in range(4):
            np.multiply(fq[sl, :n], _TET_A - _TET_B, out=share[:n])
            share[:n] += fsum[:n]
            share[:n] *= vol4[:, None]
            S = sp.csr_matrix((np.ones(n), (el[:, sl], cols)), shape=(nv, n))
            _sparsetools.csr_matvecs(nv, n, R3, S.indptr, S.indices, S.data,
                                     share[:n].ravel(), F.ravel())
    return [np.ascontiguousarray(F[:, 3 * r:3 * r + 3]) for r in range(n_rhs)]


def cfg4(n: int = 129, n_rhs: int = 16) -> Mesh:
    """3D, 129^3 jittered grid (seed 3), clamped at x=0, 16 smooth random load cases."""
    m = small3d(n, seed=3, fix="x0")
    m.rhs = load_fourier_tet(m.coords, m.elems, n_rhs)
    m.name = f"cfg4_3d_{n}cubed_{n_rhs}rhs"
    return m


def request_mesh(i: int) -> Mesh:
    """Request i of the serving stream: 2D or 3D jittered mesh, DOFs log-uniform in
    [1e3, 1e6], nu ~ U[0.25, 0.45], E in {1,100} on a random 4^d checkerboard."""
    rng = np.random.default_rng(1000 + i)
    dim = 2 if rng.random() < 0.5 else 3
    T = 10.0 ** rng.uniform(3.0, 6.0)
    nu = rng.uniform(0.25, 0.45)
    table = rng.random(4 ** dim)
    jseed = int(rng.integers(0, 2 ** 31))
    if dim == 2:
        n = max(4, int(round(np.sqrt(T / 2.0))) + 2)
        coords, el, bnd = grid2d(n, jseed)
        fixed = np.zeros((coords.shape[0], 2), dtype=np.uint8)
        fixed[bnd] = 1
        f = (0.0, -1.0)
    else:
        n = 3
        while 3 * (n - 1) * n * n < T:
            n += 1
        coords, el, bnd = grid3d(n, jseed)
        fixed = np.zeros((coords.shape[0], 3), dtype=np.uint8)
        fixed[coords[:, 0] == 0.0] = 1
        f = (0.0, 0.0, -1.0)
    cen = coords[el].mean(axis=1)
    b = np.minimum((cen * 4).astype(np.int64), 3)
    idx = b[:, 0] + 4 * b[:, 1] + (16 * b[:, 2] if dim == 3 else 0)
    E = np.where(table[idx] < 0.5, 100.0, 1.0)
    F = load_constant(coords, el, f)
    return Mesh(f"request{i}_{dim}d_n{n}", dim, coords, el, E, np.full(el.shape[0], nu), fixed, [F])
