"""P1 finite-element stiffness matrix for linear elasticity (oracle).

Test infrastructure only (see the package header).

Follows Section 2 of the paper: the problem -div sigma(u) = f with
sigma = 2 mu eps(u) + lambda tr(eps(u)) I, the weak form a(u,v) = (f,v) with
a(u,v) = int sigma(u):eps(v), the Lame constants mu = E/(2(1+nu)) and
lambda = E nu/((1+nu)(1-2nu)), and the P1 Galerkin system A U = F.

DOF numbering here is vertex-major (DOF = vertex*d + component). The paper
writes the system component-major ([U1; U2]); ``component_major_perm`` gives
the permutation between the two.

Pins (tests/test_oracle_fem.py): rigid-body kernel of dimension 3 (2D) / 6 (3D)
of the unconstrained matrix, patch test, exact symmetry, positive definiteness
after Dirichlet elimination, the paper's 2x2 operator-block form of A, and the
O(h^2) L2 convergence of a manufactured solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def lame(E, nu):
    """Lame constants (Section 2, constitutive equation)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def p1_gradients(coords: np.ndarray, elems: np.ndarray):
    """Constant gradients of the d+1 barycentric basis functions of each simplex.

    With X the d x d matrix whose row a is x_a - x_0, a point is
    x = x_0 + X^T lambda, so grad lambda_a (a >= 1) is row a of X^{-T} and
    grad lambda_0 = -sum of the others. Returns (G [Ne, d+1, d], measure [Ne]).
    """
    d = coords.shape[1]
    X = coords[elems[:, 1:]] - coords[elems[:, :1]]          # [Ne, d, d]
    det = np.linalg.det(X)
    Xinv = np.linalg.inv(X)                                    # [Ne, d, d]
    G = np.empty((elems.shape[0], d + 1, d))
    G[:, 1:, :] = np.transpose(Xinv, (0, 2, 1))
    G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
    fact = 2.0 if d == 2 else 6.0
    return G, np.abs(det) / fact


def element_stiffness(G: np.ndarray, vol: np.ndarray, mu: np.ndarray, lam: np.ndarray):
    """Element matrices K_e[(a,i),(b,j)] of a(phi_b e_j, phi_a e_i) (Section 2, weak form).

    2 mu eps(u):eps(v) + lambda div u div v with u = phi_b e_j, v = phi_a e_i gives
    mu delta_ij grad phi_a . grad phi_b + mu d_j phi_a d_i phi_b + lambda d_i phi_a d_j phi_b,
    times the element measure. Returns [Ne, (d+1)*d, (d+1)*d] in (vertex, component) order.
    """
    ne, nv, d = G.shape
    K = np.zeros((ne, nv, d, nv, d))
    GG = np.einsum("eak,ebk->eab", G, G)                     # grad phi_a . grad phi_b
    for i in range(d):
        for j in range(d):
            term = (mu[:, None, None] * np.einsum("ea,eb->eab", G[:, :, j], G[:, :, i])
                    + lam[:, None, None] * np.einsum("ea,eb->eab", G[:, :, i], G[:, :, j]))
            if i == j:
                term = term + mu[:, None, None] * GG
            K[:, :, i, :, j] = term
    K *= vol[:, None, None, None, None]
    return K.reshape(ne, nv * d, nv * d)


def assemble(coords: np.ndarray, elems: np.ndarray, E, nu) -> sp.csr_matrix:
    """Global stiffness matrix (all vertices, no boundary conditions), vertex-major."""
    nvtx, d = coords.shape
    G, vol = p1_gradients(coords, elems)
    mu, lam = lame(np.broadcast_to(E, vol.shape), np.broadcast_to(nu, vol.shape))
    Ke = element_stiffness(G, vol, mu, lam)
    dofs = (elems[:, :, None] * d + np.arange(d)[None, None, :]).reshape(elems.shape[0], -1)
    rows = np.repeat(dofs, dofs.shape[1], axis=1).ravel()
    cols = np.tile(dofs, (1, dofs.shape[1])).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(nvtx * d, nvtx * d)).tocsr()
    K.sum_duplicates()
    return K


def assemble_block_form_2d(coords: np.ndarray, elems: np.ndarray, E, nu) -> sp.csr_matrix:
    """The paper's 2x2 operator-block form of A, component-major (Section 2, system (equ)).

    A = [[lam A11 + 2mu A11 + mu A22, lam A12 + mu A21],
         [lam A21 + mu A12, lam A22 + 2mu A22 + mu A11]]
    with A_kl[a, b] = int d_k phi_a d_l phi_b. Material constants are taken per
    element. Used only as an independent check of ``assemble``.
    """
    nvtx = coords.shape[0]
    G, vol = p1_gradients(coords, elems)
    mu, lam = lame(np.broadcast_to(E, vol.shape), np.broadcast_to(nu, vol.shape))
    rows = np.repeat(elems, 3, axis=1).ravel()
    cols = np.tile(elems, (1, 3)).ravel()

    def scal(k, l, coef):
        vals = coef[:, None, None] * vol[:, None, None] * np.einsum("ea,eb->eab", G[:, :, k], G[:, :, l])
        return sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(nvtx, nvtx)).tocsr()

    B11 = scal(0, 0, lam) + scal(0, 0, 2 * mu) + scal(1, 1, mu)
    B12 = scal(0, 1, lam) + scal(1, 0, mu)
    B21 = scal(1, 0, lam) + scal(0, 1, mu)
    B22 = scal(1, 1, lam) + scal(1, 1, 2 * mu) + scal(0, 0, mu)
    return sp.bmat([[B11, B12], [B21, B22]]).tocsr()


def component_major_perm(n_vertices: int, d: int) -> np.ndarray:
    """perm such that x_cm = x_vm[perm]: component-major position a*N + v holds
    vertex-major DOF v*d + a (the paper's [U1; U2; ...] order)."""
    v = np.arange(n_vertices)
    return (v[None, :] * d + np.arange(d)[:, None]).ravel()


def free_vertices(fixed: np.ndarray) -> np.ndarray:
    """Vertices with at least one unconstrained component, ascending (their
    order is the fine level's canonical order); fully fixed vertices are
    eliminated (homogeneous Dirichlet conditions, Section 2)."""
    fixed = np.asarray(fixed).astype(bool)
    return np.flatnonzero(~fixed.all(axis=1))


def constrained_dofs(fixed: np.ndarray, free: np.ndarray) -> np.ndarray:
    """Boolean mask over the DOFs of the kept vertices (vertex-major): True for
    a fixed component of a partially constrained vertex."""
    return np.asarray(fixed).astype(bool)[free].ravel()


def restrict_free(K: sp.csr_matrix, free: np.ndarray, d: int,
                  cmask: np.ndarray | None = None) -> sp.csr_matrix:
    """Eliminate the fully fixed vertices (homogeneous Dirichlet: no lifting
    needed); a fixed component of a kept vertex (cmask) gets an identity row and
    column, which leaves the other DOFs' equations exactly those of eliminating
    it (its value is 0)."""
    dofs = (free[:, None] * d + np.arange(d)[None, :]).ravel()
    A = K[dofs][:, dofs].tocsr()
    if cmask is not None and cmask.any():
        keep = sp.diags((~cmask).astype(np.float64))
        A = (keep @ A @ keep + sp.diags(cmask.astype(np.float64))).tocsr()
        A.sort_indices()
    return A


def fine_pattern(elems: np.ndarray, free: np.ndarray, n_vertices: int) -> sp.csr_matrix:
    """Structural vertex adjacency (incl. self) among free vertices: i ~ j iff they
    share an element. Values are element counts (>0), so no entry can cancel."""
    nv1 = elems.shape[1]
    rows = np.repeat(elems, nv1, axis=1).ravel()
    cols = np.tile(elems, (1, nv1)).ravel()
    S = sp.coo_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(n_vertices, n_vertices)).tocsr()
    return S[free][:, free].tocsr()
