"""CPU tests of libvasmg: the library loads, exports every symbol of
include/vasmg.h, its host setup reproduces the oracle's hierarchy (identical
integer structure, bit-identical level-1 weights, operators to rounding), and
it rejects invalid input with the documented status codes. No GPU calls."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2505_09064_amd as pkg
from paper_2505_09064_amd import vasmg as V
from oracle import Oracle, OracleOptions
from workloads import cfg1, small2d, small3d

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "vasmg.h")


def test_library_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(vasmg_[a-z_]+)\s*\(", text))
    declared.discard("vasmg_ctx")
    lib = pkg.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(pkg.EXPORTED)


def _compare(mesh, oopts=None, **kw):
    oopts = oopts or OracleOptions()
    o = Oracle(mesh.coords, mesh.elems, mesh.E, mesh.nu, mesh.fixed, oopts)
    s = V.Solver.from_mesh(mesh, host_only=1, **kw)
    nl, nd, dim = s.hierarchy_info()
    assert nl == o.L + 1
    assert nd == o.A[0].shape[0]
    d = mesh.dim
    m, M, depth = s.tree_info()
    assert depth == o.levels.max_depth
    assert (m, M) == (o.levels.m, o.levels.M)
    for l in range(nl):
        e = s.export_level(l)
        n = e["n_vertices"]
        A = sp.bsr_matrix((e["vals"], e["cols"], e["rowptr"]), shape=(n * d, n * d)).tocsr()
        assert abs(A - o.A[l]).max() <= 1e-13 * abs(o.A[l]).max()
        S = sp.csr_matrix((np.ones(e["cols"].size), e["cols"], e["rowptr"]), shape=(n, n))
        assert (S != (o.S[l] > 0)).nnz == 0, "structural pattern differs"
        if l < o.L:
            assert np.array_equal(e["cell"], o.cells[l])
            assert np.array_equal(e["block"], o.blocks[l])
            assert np.array_equal(e["color"], o.colors[l])
            assert e["n_colors"] == o.colors[l].max() + 1
            P = sp.csr_matrix((e["p_vals"], e["p_cols"], e["p_rowptr"]), shape=o.P[l].shape)
            diff = P - o.P[l]
            assert diff.nnz == 0 or abs(diff).max() == 0.0, "P not bit-identical"
        if l >= 1:
            assert np.array_equal(e["keys"], o.levels.level_keys(l))
        # constrained components (bit a = component a) against the oracle's mask
        bits = np.zeros(n, dtype=np.uint8)
        for a in range(d):
            bits |= (o.cmask[l].reshape(n, d)[:, a].astype(np.uint8) << a)
        assert np.array_equal(e["fixed"], bits), l
    s.free()


@pytest.mark.parametrize("name", ["cfg1", "small3d", "small2d_x0", "graded", "cap9", "free_tree",
                                  "truncated", "mixed_material", "symmetry2d", "symmetry3d",
                                  "clamp_rollers3d", "symmetry3d_color_blocks", "symmetry3d_free_tree",
                                  "small3d_color_blocks"])
def test_host_setup_matches_oracle(name):
    if name == "cfg1":
        _compare(cfg1())
    elif name == "small3d":
        _compare(small3d(9, seed=5))
    elif name == "small2d_x0":
        _compare(small2d(17, seed=3, fix="x0"))
    elif name == "graded":
        _compare(small2d(33, seed=None, graded=True, nu=0.49))
    elif name == "cap9":
        _compare(small2d(17, seed=4), OracleOptions(leaf_capacity=9), leaf_capacity=9)
    elif name == "free_tree":
        _compare(small3d(7, seed=6), OracleOptions(tree_vertices="free"), tree_vertices=V.TREE_FREE)
    elif name == "truncated":
        _compare(small2d(21, seed=7), OracleOptions(coarsest_max_dofs=300), coarsest_max_dofs=300)
    elif name == "mixed_material":
        m = small3d(8, seed=9)
        rng = np.random.default_rng(0)
        m.E = np.where(rng.random(m.elems.shape[0]) < 0.5, 1.0, 100.0)
        m.nu = rng.uniform(0.25, 0.45, m.elems.shape[0])
        _compare(m)
    elif name == "symmetry2d":
        _compare(small2d(17, seed=2, fix="symmetry"))
    elif name == "symmetry3d":
        _compare(small3d(9, seed=5, fix="symmetry"))
    elif name == "clamp_rollers3d":
        _compare(small3d(7, seed=3, fix="roller_x1"))
    elif name == "small3d_color_blocks":
        _compare(small3d(9, seed=5), OracleOptions(color_blocks="auto"), color_blocks=1)
    elif name == "symmetry3d_color_blocks":
        _compare(small3d(9, seed=5, fix="symmetry"), OracleOptions(color_blocks="auto"),
                 color_blocks=1)
    elif name == "symmetry3d_free_tree":
        _compare(small3d(9, seed=5, fix="symmetry"), OracleOptions(tree_vertices="free"),
                 tree_vertices=V.TREE_FREE)


def _expect(status, mesh_fn, **kw):
    m = mesh_fn()
    with pytest.raises(V.VasmgError) as ei:
        V.Solver.from_mesh(m, host_only=1, **kw)
    assert ei.value.status == status, str(ei.value)
    return str(ei.value)


def test_setup_rejects_invalid_input():
    def bad_flag():
        m = small2d(5); m.fixed[7, 0] = 2; return m

    def inverted():
        m = small2d(5); m.elems[3, [1, 2]] = m.elems[3, [2, 1]]; return m

    def bad_nu():
        m = small2d(5); m.nu = np.full(m.elems.shape[0], 0.5); return m

    def bad_E():
        m = small2d(5); m.E = np.zeros(m.elems.shape[0]); return m

    def bad_index():
        m = small2d(5); m.elems[0, 0] = m.n_vertices; return m

    def nan_coord():
        m = small2d(5); m.coords[4, 1] = np.nan; return m

    def all_fixed():
        m = small2d(5); m.fixed[:] = 1; return m

    def duplicates():
        m = small2d(5)
        m.coords = np.concatenate([m.coords, np.repeat(m.coords[12:13], 6, 0)])
        m.fixed = np.concatenate([m.fixed, np.ones((6, 2), np.uint8)])
        return m

    for fn in (bad_flag, inverted, bad_nu, bad_E, bad_index, nan_coord, all_fixed, duplicates):
        _expect(V.EINVAL, fn)
    _expect(V.EDEGENERATE, lambda: small2d(6, fix="none"))
    # one free vertex interpolated from 2^d coarse corners: a rank-d coarsest
    # operator, refused by the oracle as well
    for one_free in (lambda: small2d(3, seed=1, fix="boundary"), lambda: small3d(3, seed=1, fix="boundary")):
        _expect(V.EDEGENERATE, one_free)
        m = one_free()
        with pytest.raises(np.linalg.LinAlgError):
            Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    _expect(V.EINVAL, lambda: small2d(5), leaf_capacity=-1)
    _expect(V.EINVAL, lambda: small2d(5), block_rhs=5)
    _expect(V.EINVAL, lambda: small2d(5), block_rhs=4, block_lanes=3)
    _expect(V.EINVAL, lambda: small2d(5), block_lanes=-1)


def test_host_only_handle_refuses_device_calls():
    m = small2d(5)
    s = V.Solver.from_mesh(m, host_only=1)
    with pytest.raises(V.VasmgError) as ei:
        s.solve(m.rhs[0])
    assert ei.value.status == V.EDEVICE
    s.free()
    s.free()   # idempotent


def test_default_options():
    o = V.default_options(2)
    assert (o.leaf_capacity, o.n_pre, o.n_post, o.max_iters) == (4, 1, 1, 10000)
    assert V.default_options(3).leaf_capacity == 8
    assert o.block_rhs == 0 and o.block_lanes == 0
    with pytest.raises(V.VasmgError):
        V.default_options(4)


def test_server_default_config():
    """The documented server defaults (no device needed to read them): 4 slots, 4
    setup workers, 80% of free memory, packing off, and the host-setup size limits
    of 131,072 DOFs in 2D and 16,384 in 3D."""
    cfg = V.ServerConfig()
    V._check(V.lib().vasmg_server_default_config(V.C.byref(cfg)))
    assert (cfg.slots, cfg.setup_workers, cfg.hbm_budget_bytes) == (4, 4, 0)
    assert (cfg.pack_max_dofs, cfg.pack_max_parts, cfg.pack_wait_ms) == (0, 16, 0)
    assert (cfg.host_setup_max_dofs_2d, cfg.host_setup_max_dofs_3d) == (131072, 16384)
    assert cfg.options.leaf_capacity == 0 and cfg.options.n_pre == 1
    assert V.lib().vasmg_server_default_config(None) == V.EINVAL


def test_device_bytes_estimate_and_no_device_paths():
    import torch
    m = small3d(7, seed=2)
    s = V.Solver.from_mesh(m, host_only=1)
    b = V.C.c_int64()
    V._check(V.lib().vasmg_device_bytes(s._h, V.C.byref(b)))
    A = s.export_level(0)
    assert b.value > 8 * 9 * len(A["cols"])          # at least the fine FP64 blocks
    if not torch.cuda.is_available():
        assert V.lib().vasmg_upload(s._h, None) == V.EDEVICE
        with pytest.raises(V.VasmgError) as ei:
            V.Server(slots=1, setup_workers=1)
        assert ei.value.status == V.EDEVICE
    s.free()


def test_setup_device_option_validation():
    """setup_device takes 0 or 1 (EINVAL otherwise, checked before any device
    call); without a device setup_device = 1 fails with EDEVICE, also host-only;
    the Galerkin window hook rejects negative sizes and restores the default."""
    import torch
    m = small2d(9, seed=1)
    with pytest.raises(V.VasmgError) as ei:
        V.Solver.from_mesh(m, host_only=1, setup_device=3)
    assert ei.value.status == V.EINVAL
    assert V.default_options(3).setup_device == 0
    if not torch.cuda.is_available():
        for kw in (dict(setup_device=1), dict(setup_device=1, host_only=1)):
            with pytest.raises(V.VasmgError) as ei:
                V.Solver.from_mesh(m, **kw)
            assert ei.value.status == V.EDEVICE
    with pytest.raises(V.VasmgError) as ei:
        V.set_galerkin_window(-5)
    assert ei.value.status == V.EINVAL
    V.set_galerkin_window(0)


def test_binding_refuses_tensors_it_cannot_pass_safely():
    """The binding checks device tensors before handing their pointers to the
    kernels (which index them by the handle's sizes)."""
    torch = pytest.importorskip("torch")
    from paper_2505_09064_amd.vasmg import _check_tensor
    with pytest.raises(ValueError, match="HIP device"):
        _check_tensor(torch.zeros((4, 3), dtype=torch.float64), (4, 3), "d_x")
    with pytest.raises(ValueError, match="torch tensor"):
        _check_tensor(np.zeros((4, 3)), (4, 3), "d_x")
    with pytest.raises(ValueError, match="torch tensor"):
        _check_tensor(None, (4, 3), "d_x")


def test_setup_phases_of_a_host_setup():
    """vasmg_setup_phases reports the host setup's phases in the order they ran
    (the host tree and prolongations, then the products and the ordering), with
    non-negative wall-clock times; a partially constrained mesh adds the coarse
    constraint phase."""
    s = V.Solver.from_mesh(small3d(7, seed=2), host_only=1)
    ph = s.setup_phases()
    assert [n for n, _ in ph] == ["validate+assemble", "tree", "P0", "coarse regions+P", "galerkin",
                                  "cells+colours", "coarsest factor"]
    assert all(ms >= 0.0 for _, ms in ph)
    s.free()
    s = V.Solver.from_mesh(small3d(7, seed=3, fix="roller_x1"), host_only=1)
    assert "coarse constraints" in [n for n, _ in s.setup_phases()]
    s.free()
