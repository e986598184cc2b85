"""Packing on the host (vasmg_pack of host-only handles; no GPU calls).

The packed hierarchy must be exactly the block-diagonal union of the parts':
level l holds every part's level min(l, L_i) (a shallower part repeats its
coarsest level, joined to the next copy by an identity prolongation), operators
and prolongations bit for bit, each part's Gauss-Seidel order kept (its cells
renumbered after the previous parts', its colours unchanged; a repeated
coarsest level swept point by point, or as one cell when it has at most 2^d
vertices), constrained components carried along, and the user vertices of the
parts one after the other. Packing rejects parts it cannot serve."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2505_09064_amd import vasmg as V
from workloads import small2d, small3d


def _bsr(e, d):
    n = e["n_vertices"]
    return sp.bsr_matrix((e["vals"], e["cols"], e["rowptr"]), shape=(n * d, n * d)).tocsr()


def _P(e, ncols):
    return sp.csr_matrix((e["p_vals"], e["p_cols"], e["p_rowptr"]), shape=(e["n_vertices"], ncols))


PACKS = {
    # different depths (5 and 17 points per side), a symmetry-plane part, a graded part
    "2d": lambda: [small2d(5, seed=1), small2d(17, seed=2, fix="symmetry"), small2d(9, seed=3),
                   small2d(17, seed=None, graded=True, nu=0.49)],
    "3d": lambda: [small3d(5, seed=1), small3d(7, seed=2, fix="roller_x1"), small3d(4, seed=3)],
}


@pytest.mark.parametrize("name", list(PACKS))
def test_packed_hierarchy_is_the_block_diagonal_union(name):
    meshes = PACKS[name]()
    d = meshes[0].dim
    parts = [V.Solver.from_mesh(m, host_only=1) for m in meshes]
    depth = [p.hierarchy_info()[0] for p in parts]
    assert len(set(depth)) > 1, "the pack should mix depths"
    pk = V.PackedSolver(parts, upload=False)
    nl, ndof, dim = pk.hierarchy_info()
    assert nl == max(depth) and dim == d
    assert ndof == sum(p.hierarchy_info()[1] for p in parts)
    assert list(pk.offsets) == list(np.cumsum([0] + [m.n_vertices for m in meshes]))
    for l in range(nl):
        src = [min(l, n - 1) for n in depth]
        e = pk.export_level(l)
        ep = [p.export_level(s) for p, s in zip(parts, src)]
        A = _bsr(e, d)
        Ab = sp.block_diag([_bsr(x, d) for x in ep], format="csr")
        assert A.shape == Ab.shape and (A != Ab).nnz == 0, l
        assert np.array_equal(e["fixed"], np.concatenate([x["fixed"] for x in ep])), l
        if l == nl - 1:
            continue
        # prolongation: each part's own, or the identity below its depth
        nxt = [min(l + 1, n - 1) for n in depth]
        blocks = []
        for p, x, s, t in zip(parts, ep, src, nxt):
            if t > s:
                blocks.append(_P(x, p.level_info(t)["n_vertices"]))
            else:
                blocks.append(sp.identity(x["n_vertices"], format="csr"))
        Pb = sp.block_diag(blocks, format="csr")
        assert (_P(e, Pb.shape[1]) != Pb).nnz == 0, l
        # Gauss-Seidel order: a part's own where it has the level, point order below
        off_v, off_c = 0, 0
        for x, s, n in zip(ep, src, depth):
            nv = x["n_vertices"]
            cell = e["cell"][off_v:off_v + nv]
            color = e["color"][off_v:off_v + nv]
            if s < n - 1:
                assert np.array_equal(cell, x["cell"] + off_c), (l, "cells")
                assert np.array_equal(color, x["color"]), (l, "colours")
                off_c += int(x["cell"].max()) + 1
            else:
                if l > 0 and nv <= (1 << d):
                    assert np.all(cell == off_c) and np.all(color == 0)
                    off_c += 1
                else:
                    assert np.array_equal(cell, off_c + np.arange(nv))
                    off_c += nv
                    # a proper colouring of the padded level's couplings
                    S = sp.csr_matrix((np.ones(x["cols"].size), x["cols"], x["rowptr"]),
                                      shape=(nv, nv)).tocoo()
                    off = S.row != S.col
                    assert np.all(color[S.row[off]] != color[S.col[off]])
            off_v += nv
        assert e["n_colors"] == int(e["color"].max()) + 1
    pk.free()
    for p in parts:
        p.free()


def test_pack_rejects_what_it_cannot_serve():
    a, b = small2d(5, seed=1), small3d(4, seed=2)
    pa = V.Solver.from_mesh(a, host_only=1)
    pb = V.Solver.from_mesh(b, host_only=1)
    for parts, why in (([pa, pb], "dimension"),
                       ([pa, V.Solver.from_mesh(a, host_only=1, precision=V.FP32_PRECOND)], "precision"),
                       ([pa, V.Solver.from_mesh(a, host_only=1, cycle=V.CYCLE_W)], "cycle"),
                       ([pb, V.Solver.from_mesh(b, host_only=1, color_blocks=1)], "colour blocks"),
                       ([pa, V.Solver.from_mesh(a, host_only=1, smoother=V.SMOOTHER_JACOBI)], "smoother")):
        with pytest.raises(V.VasmgError) as ei:
            V.PackedSolver(parts, upload=False)
        assert ei.value.status == V.EINVAL, why
    with pytest.raises(ValueError):
        V.PackedSolver([], upload=False)
    # a packed handle solves only through the packed entry points, and only on a device
    pk = V.PackedSolver([pa, V.Solver.from_mesh(a, host_only=1)], upload=False)
    with pytest.raises(V.VasmgError) as ei:
        pk.solve_packed([a.rhs[0], a.rhs[0]])
    assert ei.value.status == V.EDEVICE
    assert [n for n, _ in pk.setup_phases()] == ["pack"]
