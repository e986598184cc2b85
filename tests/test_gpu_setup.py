"""GPU tests of the device setup (setup_device = 1): the fine assembly and the
coarse operators A_{l+1} = P_l^T A_l P_l of Section 3 formed on the device.

Parity bars: against the oracle's hierarchy the same as the host setup's (the
column structure identical, values within 1e-13 of the largest entry of the
level); against the host setup, identical integer structure (columns, cells,
colours, keys, P), the fine level bit for bit and the coarse values to rounding; between device setups, bitwise
equality (the numeric pass sums in a fixed order, independent of the launch and
of the bitmap window). Solves from a device-built hierarchy take the iteration
counts of the host-built one.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Oracle, OracleOptions
from oracle.smoother import ColoredGS
from workloads import cfg1, small2d, small3d

torch = pytest.importorskip("torch")
from paper_2505_09064_amd import vasmg as V  # noqa: E402

pytestmark = pytest.mark.gpu


def _levels(s):
    nl, _, _ = s.hierarchy_info()
    return [s.export_level(l) for l in range(nl)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _bsr(e, d):
    n = e["n_vertices"]
    return sp.bsr_matrix((e["vals"], e["cols"], e["rowptr"]), shape=(n * d, n * d)).tocsr()


CASES = {
    "cfg1": (cfg1, {}, OracleOptions()),
    "small3d": (lambda: small3d(9, seed=5), {}, OracleOptions()),
    "small2d_x0": (lambda: small2d(17, seed=3, fix="x0"), {}, OracleOptions()),
    "graded": (lambda: small2d(33, seed=None, graded=True, nu=0.49), {}, OracleOptions()),
    "cap9": (lambda: small2d(17, seed=4), {"leaf_capacity": 9}, OracleOptions(leaf_capacity=9)),
    "free_tree": (lambda: small3d(7, seed=6), {"tree_vertices": V.TREE_FREE},
                  OracleOptions(tree_vertices="free")),
    "truncated": (lambda: small2d(21, seed=7), {"coarsest_max_dofs": 300},
                  OracleOptions(coarsest_max_dofs=300)),
    "symmetry3d": (lambda: small3d(9, seed=5, fix="symmetry"), {}, OracleOptions()),
    "clamp_rollers3d": (lambda: small3d(7, seed=3, fix="roller_x1"), {}, OracleOptions()),
}


@pytest.mark.parametrize("name", list(CASES))
def test_device_galerkin_matches_oracle_and_host(name):
    mesh_fn, kw, oopts = CASES[name]
    m = mesh_fn()
    d = m.dim
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, oopts)
    sd = V.Solver.from_mesh(m, setup_device=1, **kw)
    sh = V.Solver.from_mesh(m, host_only=1, **kw)
    Ld, Lh = _levels(sd), _levels(sh)
    assert len(Ld) == len(Lh) == o.L + 1
    for l, (ed, eh) in enumerate(zip(Ld, Lh)):
        for key in ("rowptr", "cols", "cell", "block", "color", "fixed", "keys", "p_rowptr",
                    "p_cols", "p_vals"):
            if ed.get(key) is not None:
                assert np.array_equal(ed[key], eh[key]), (l, key)
        Ad = _bsr(ed, d)
        scale = abs(o.A[l]).max()
        assert abs(Ad - o.A[l]).max() <= 1e-13 * scale, l
        assert np.abs(ed["vals"] - eh["vals"]).max() <= 1e-13 * scale, l
        S = sp.csr_matrix((np.ones(ed["cols"].size), ed["cols"], ed["rowptr"]),
                          shape=(ed["n_vertices"],) * 2)
        assert (S != (o.S[l] > 0)).nnz == 0, "structural pattern differs from the oracle"
    # the device assembly follows the host's arithmetic: the same fine values bit for bit
    assert np.array_equal(Ld[0]["vals"], Lh[0]["vals"])
    # the tree, keys and prolongations came from the device build
    assert "tree+P (device)" in [n for n, _ in sd.setup_phases()]
    assert "tree" in [n for n, _ in sh.setup_phases()]
    assert sd.tree_info() == sh.tree_info()
    sd.free()
    sh.free()


def _compare_transfers(sd, sh):
    """Device- and host-built trees, keys and prolongations: identical."""
    assert sd.tree_info() == sh.tree_info()
    Ld, Lh = _levels(sd), _levels(sh)
    assert len(Ld) == len(Lh)
    for l, (ed, eh) in enumerate(zip(Ld, Lh)):
        for key in ("keys", "p_rowptr", "p_cols", "p_vals", "cell", "color", "rowptr", "cols"):
            if eh.get(key) is not None:
                assert np.array_equal(ed[key], eh[key]), (l, key)


@pytest.mark.parametrize("name", ["cube33_3d", "graded129_2d", "cube33_3d_free_tree"])
def test_device_tree_matches_host_at_size(name):
    """The device tree build (level-synchronous rounds, packed lattice keys)
    at sizes with many rounds, large sorts and deep graded trees: the same root
    box, depth, level keys and prolongations (structure and weights bit for bit)
    as the host build, whose own output is pinned to the oracle's."""
    kw = {"tree_vertices": V.TREE_FREE} if name.endswith("free_tree") else {}
    m = small2d(129, seed=None, graded=True, nu=0.49) if name.startswith("graded") else \
        small3d(33, seed=1, fix="x0")
    sd = V.Solver.from_mesh(m, setup_device=1, host_only=1, **kw)
    sh = V.Solver.from_mesh(m, host_only=1, **kw)
    assert "tree+P (device)" in [n for n, _ in sd.setup_phases()]
    _compare_transfers(sd, sh)
    sd.free()
    sh.free()


def _random_tree_mesh(i):
    rng = np.random.default_rng(7000 + i)
    dim = int(rng.integers(2, 4))
    tie = rng.random() < 0.3          # no jitter, 2^k + 1 vertices: points on midlines
    if dim == 2:
        n = int(2 ** rng.integers(2, 7) + 1) if tie else int(rng.integers(4, 90))
        m = small2d(n, seed=None if tie else int(rng.integers(0, 1000)),
                    fix=str(rng.choice(["boundary", "x0", "symmetry"])))
    else:
        n = int(2 ** rng.integers(2, 5) + 1) if tie else int(rng.integers(3, 26))
        m = small3d(n, seed=None if tie else int(rng.integers(0, 1000)),
                    fix=str(rng.choice(["x0", "symmetry", "roller_x1"])))
    if rng.random() < 0.5:            # clustered points: monotone per-axis maps
        m.coords = m.coords ** rng.uniform(0.4, 3.0, size=dim)
    cap = int(rng.choice([0, 0, 0, 1, 2, 3, 5, 9, 12, 27]))
    tv = V.TREE_FREE if rng.random() < 0.3 else V.TREE_ALL
    return m, cap, tv


@pytest.mark.parametrize("i", range(30))
def test_device_tree_matches_host_random(i):
    """Seeded random meshes (clustered points, vertices exactly on midlines, leaf
    capacities 1 to 27, all or free tree vertices): the device tree build gives the
    host's root box, depth, keys, prolongations, cells, colours and operator
    patterns bit for bit."""
    m, cap, tv = _random_tree_mesh(i)
    sh = V.Solver.from_mesh(m, host_only=1, leaf_capacity=cap, tree_vertices=tv)
    sd = V.Solver.from_mesh(m, host_only=1, setup_device=1, leaf_capacity=cap, tree_vertices=tv)
    assert "tree+P (device)" in [n for n, _ in sd.setup_phases()]
    _compare_transfers(sd, sh)
    sd.free()
    sh.free()


@pytest.mark.parametrize("dim", [2, 3])
def test_device_tree_falls_back_to_host_when_too_deep(dim):
    """A leaf's capacity of fixed vertices within 2^-44 (2D) / 2^-30 (3D) of
    the box of another vertex need a tree deeper than packed keys allow (32 / 21
    levels): the device build declines, the host builds it, and the result
    equals a host setup's."""
    m = small2d(7, seed=2) if dim == 2 else small3d(5, seed=2)
    eps = 2.0 ** -44 if dim == 2 else 2.0 ** -30
    cap = 4 if dim == 2 else 8
    extra = m.coords[12:13] + eps * np.arange(1, cap + 1)[:, None]
    m.coords = np.concatenate([m.coords, extra])
    m.fixed = np.concatenate([m.fixed, np.ones((cap, dim), np.uint8)])
    sd = V.Solver.from_mesh(m, setup_device=1, host_only=1)
    sh = V.Solver.from_mesh(m, host_only=1)
    names = [n for n, _ in sd.setup_phases()]
    assert "tree" in names and "tree+P (device)" not in names
    assert sd.tree_info()[2] > (32 if dim == 2 else 21)
    _compare_transfers(sd, sh)
    sd.free()
    sh.free()


@pytest.mark.parametrize("name", ["small3d", "small2d_x0", "graded", "symmetry3d"])
@pytest.mark.parametrize("prec", [V.FP64, V.FP32_PRECOND])
def test_device_layout_kernels_per_level(name, prec):
    """The level layouts built on the device (colour-ordered rows, sorted and
    quad-padded L / U parts, cell matrices or diagonals) drive the per-level
    kernels to the oracle's results with the bars of the host-built layouts, and
    on the fine level (assembled on the host, so the same FP64 values) to the
    host-built layout's results bit for bit."""
    mesh_fn, kw, oopts = CASES[name]
    m = mesh_fn()
    d = m.dim
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, oopts)
    sd = V.Solver.from_mesh(m, precision=prec, setup_device=1, **kw)
    sh = V.Solver.from_mesh(m, precision=prec, **kw)
    rng = np.random.default_rng(4)
    tol = 1e-13 if prec == V.FP64 else 2e-6
    gtol = 1e-11 if prec == V.FP64 else 1e-4
    for l in range(o.L):
        A = o.A[l]
        n = A.shape[0] // d
        x = rng.normal(size=(n, d))
        b = rng.normal(size=(n, d))
        yd = torch.zeros((n, d), dtype=torch.float64, device="cuda")
        yh = torch.zeros_like(yd)
        sd.spmv_device(l, prec, _dev(x), yd)
        sh.spmv_device(l, prec, _dev(x), yh)
        assert _rel(_host(yd).ravel(), A @ x.ravel()) < tol, (l, "spmv")
        if l == 0:
            assert np.array_equal(_host(yd), _host(yh)), "fine SpMV not bitwise equal"
        S = o.gs(l)
        for bw in (0, 1):
            xd, xh = _dev(x), _dev(x)
            sd.gs_sweep_device(l, prec, bw, _dev(b), xd)
            sh.gs_sweep_device(l, prec, bw, _dev(b), xh)
            ref = S.backward(b.ravel(), x.ravel()) if bw else S.forward(b.ravel(), x.ravel())
            assert _rel(_host(xd).ravel(), ref) < gtol, (l, "gs", bw)
            if l == 0:
                assert np.array_equal(_host(xd), _host(xh)), ("fine GS not bitwise equal", bw)
    sd.free()
    sh.free()


@pytest.mark.parametrize("kw", [dict(smoother=V.SMOOTHER_JACOBI), dict(block_rhs=8),
                                dict(cycle=V.CYCLE_W), dict(preconditioner=V.PRECOND_JACOBI)])
def test_device_setup_with_other_options(kw):
    """Options that read the host copies of the level values (the Jacobi
    smoother's diagonal inverses and eigenvalue estimate) or other device paths
    (block right-hand sides, W-cycle, point Jacobi preconditioner) give the
    host-setup handle's iteration counts."""
    m = small3d(9, seed=5)
    rng = np.random.default_rng(3)
    n_rhs = 3 if "block_rhs" in kw else 1
    F = rng.normal(size=(n_rhs, m.coords.shape[0], 3)) * (1 - m.fixed)[None]
    sd = V.Solver.from_mesh(m, setup_device=1, **kw)
    sh = V.Solver.from_mesh(m, **kw)
    Xd, infd = sd.solve(F, 1e-8)
    Xh, infh = sh.solve(F, 1e-8)
    for a, b in zip(infd, infh):
        assert a["converged"] == 1 and a["iterations"] == b["iterations"]
    assert np.linalg.norm(Xd - Xh) / np.linalg.norm(Xh) < 1e-7
    sd.free()
    sh.free()


def test_device_galerkin_deterministic_and_window_independent():
    """Two device setups agree bit for bit, and so does a setup whose symbolic
    pass covers 32 (then 96) columns at a time, so that every coarse row takes
    several bitmap windows."""
    m = small3d(9, seed=5)
    ref = _levels(V.Solver.from_mesh(m, setup_device=1))
    again = _levels(V.Solver.from_mesh(m, setup_device=1))
    try:
        for cols in (32, 96):
            V.set_galerkin_window(cols)
            win = _levels(V.Solver.from_mesh(m, setup_device=1))
            for a, b, c in zip(ref, again, win):
                for key in ("rowptr", "cols", "vals"):
                    assert np.array_equal(a[key], b[key]), key
                    assert np.array_equal(a[key], c[key]), (cols, key)
    finally:
        V.set_galerkin_window(0)


@pytest.mark.parametrize("precision", [V.FP64, V.FP32_PRECOND])
def test_device_galerkin_solve_matches_host_setup(precision):
    m = small3d(9, seed=5)
    rng = np.random.default_rng(2)
    F = rng.normal(size=(m.coords.shape[0], 3)) * (1 - m.fixed)
    rtol = 1e-8 if precision == V.FP64 else 1e-6
    sd = V.Solver.from_mesh(m, precision=precision, setup_device=1)
    sh = V.Solver.from_mesh(m, precision=precision)
    xd, idv = sd.solve(F, rtol)
    xh, ih = sh.solve(F, rtol)
    assert idv["converged"] == 1 and idv["rel_res_true"] < rtol
    assert idv["iterations"] == ih["iterations"]
    assert np.linalg.norm(xd - xh) / np.linalg.norm(xh) < 10 * rtol
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    xo, io = o.solve(F, rtol)
    assert abs(idv["iterations"] - io["iterations"]) <= 1
    sd.free()
    sh.free()


def test_device_galerkin_rejected_configurations():
    m = small2d(9, seed=1)
    with pytest.raises(V.VasmgError) as ei:
        V.Solver.from_mesh(m, setup_device=2)
    assert ei.value.status == V.EINVAL
    with pytest.raises(V.VasmgError):
        V.set_galerkin_window(-1)


def test_device_galerkin_host_only_then_upload():
    """setup_device = 1 with host_only = 1 (a server's setup workers): the products
    are formed on the device and brought back whole; the host-only handle equals
    the device-resident one bit for bit, and after vasmg_upload solves the same."""
    m = small3d(9, seed=5)
    sh = V.Solver.from_mesh(m, setup_device=1, host_only=1)
    sd = V.Solver.from_mesh(m, setup_device=1)
    for a, b in zip(_levels(sh), _levels(sd)):
        for key in ("rowptr", "cols", "vals", "p_cols", "p_vals"):
            assert np.array_equal(a[key], b[key]), key
    V._check(V.lib().vasmg_upload(sh._h, None))
    rng = np.random.default_rng(8)
    F = rng.normal(size=(m.coords.shape[0], 3)) * (1 - m.fixed)
    xh, ih = sh.solve(F, 1e-8)
    xd, idv = sd.solve(F, 1e-8)
    assert ih["iterations"] == idv["iterations"]
    assert np.array_equal(xh, xd)
    sh.free()
    sd.free()


def test_full_size_device_galerkin_matches_host():
    """The 65^3 workload (811,200 DOFs; level 1 holds 27.7 M blocks): the device
    hierarchy has the host's structure on every level and its values to
    rounding; the mixed-precision solve takes the same iterations."""
    import time
    from workloads import cfg2
    m = cfg2()
    t0 = time.perf_counter()
    sd = V.Solver.from_mesh(m, precision=V.FP32_PRECOND, setup_device=1)
    t1 = time.perf_counter()
    sh = V.Solver.from_mesh(m, precision=V.FP32_PRECOND)
    t2 = time.perf_counter()
    print(f"setup: device Galerkin {t1 - t0:.2f} s, host {t2 - t1:.2f} s")
    nl = sd.hierarchy_info()[0]
    assert nl == sh.hierarchy_info()[0]
    for l in range(1, nl):
        ed, eh = sd.export_level(l), sh.export_level(l)
        assert np.array_equal(ed["rowptr"], eh["rowptr"]) and np.array_equal(ed["cols"], eh["cols"])
        assert np.array_equal(ed["color"], eh["color"])
        scale = np.abs(eh["vals"]).max()
        assert np.abs(ed["vals"] - eh["vals"]).max() <= 1e-13 * scale, l
        del ed, eh
    F = m.rhs[0]
    _, idv = sd.solve(F, 1e-6)
    _, ih = sh.solve(F, 1e-6)
    assert idv["converged"] == 1 and idv["iterations"] == ih["iterations"]
    sd.free()
    sh.free()


def test_full_size_graded_2d_device_setup():
    """The graded nearly incompressible 2D workload (1025^2 vertices, nu = 0.49,
    2,093,058 DOFs, 20 levels, levels 1-9 near 1 M DOFs each) built with the
    device Galerkin products (2D kernels at full size): every level's structure
    equals the host build's, values within 1e-13 of the level's largest entry,
    and the FP64 solve meets the stored oracle values (iterations +-1, sampled
    solution within 1e-8 of max |x|)."""
    import json
    import os
    from workloads import cfg3
    path = os.path.join(os.path.dirname(__file__), "golden", "cfg3_oracle.json")
    g = json.load(open(path))
    m = cfg3()
    sd = V.Solver.from_mesh(m, precision=V.FP64, setup_device=1)
    sh = V.Solver.from_mesh(m, host_only=1)
    nl = sd.hierarchy_info()[0]
    assert nl == sh.hierarchy_info()[0]
    for l in range(1, nl):
        ed, eh = sd.export_level(l), sh.export_level(l)
        assert np.array_equal(ed["rowptr"], eh["rowptr"]) and np.array_equal(ed["cols"], eh["cols"])
        assert np.array_equal(ed["color"], eh["color"])
        scale = np.abs(eh["vals"]).max()
        assert np.abs(ed["vals"] - eh["vals"]).max() <= 1e-13 * scale, l
        del ed, eh
    sh.free()
    x, info = sd.solve(m.rhs[0], 1e-6)
    idx = np.array(g["sample_vertices"])
    print("cfg3 fp64, device setup:", info["iterations"], "its; oracle", g["fp64"]["iterations"])
    assert abs(info["iterations"] - g["fp64"]["iterations"]) <= 1
    assert np.abs(x[idx] - np.array(g["sample_x"])).max() <= 1e-8 * g["x_norminf"]
    sd.free()


def test_device_setup_background_downloads():
    """After a device setup the FP64 level values reach the host in the
    background: a handle freed at once (downloads in flight) releases cleanly, a
    solve runs while they arrive, and an export waits for them and returns the
    values of a second, settled handle bit for bit."""
    m = small3d(11, seed=7)
    for _ in range(3):
        V.Solver.from_mesh(m, setup_device=1).free()
    a = V.Solver.from_mesh(m, setup_device=1)
    x, info = a.solve(m.rhs[0], 1e-8)
    assert info["converged"] == 1
    b = V.Solver.from_mesh(m, setup_device=1)
    la = _levels(a)
    lb = _levels(b)
    for ea, eb in zip(la, lb):
        assert np.array_equal(ea["vals"], eb["vals"])
    a.free()
    b.free()


@pytest.mark.parametrize("dim", [2, 3])
def test_device_setup_single_level(dim):
    """A hierarchy truncated to the fine level (coarsest_max_dofs above its DOFs):
    the coarsest factor then needs the device-assembled fine values on the host at
    once; the solve (one V-cycle = the exact solve) matches the host setup's."""
    m = small2d(9, seed=2) if dim == 2 else small3d(4, seed=2)
    kw = dict(coarsest_max_dofs=4000)
    sd = V.Solver.from_mesh(m, setup_device=1, **kw)
    sh = V.Solver.from_mesh(m, **kw)
    assert sd.hierarchy_info()[0] == 1 == sh.hierarchy_info()[0]
    assert np.array_equal(sd.export_level(0)["vals"], sh.export_level(0)["vals"])
    xd, idv = sd.solve(m.rhs[0], 1e-10)
    xh, ih = sh.solve(m.rhs[0], 1e-10)
    assert idv["iterations"] == ih["iterations"] <= 2
    assert np.array_equal(xd, xh)
    sd.free()
    sh.free()


@pytest.mark.parametrize("name", ["small3d", "symmetry3d", "graded", "small2d_x0"])
@pytest.mark.parametrize("prec", [V.FP64, V.FP32_PRECOND])
def test_device_numbered_transfers_equal_host_built(name, prec):
    """With setup_device = 1 the upload renumbers and transposes each level's
    prolongation on the device (from the canonical P kept after the level's
    Galerkin product): restriction and prolongation through those arrays give
    the results of the host-built arrays bit for bit, on every level, in the
    handle's precision."""
    m = CASES[name][0]()
    sd = V.Solver.from_mesh(m, setup_device=1, precision=prec, autotune=0)
    sh = V.Solver.from_mesh(m, setup_device=0, precision=prec, autotune=0)
    nl = sd.hierarchy_info()[0]
    assert nl == sh.hierarchy_info()[0] and nl >= 3
    rng = np.random.default_rng(3)
    for l in range(nl - 1):
        for p in (prec,):
            r = _dev(rng.normal(size=sd._level_shape(l)))
            e = _dev(rng.normal(size=sd._level_shape(l + 1)))
            outs = []
            for s in (sd, sh):
                bc = torch.zeros(s._level_shape(l + 1), dtype=torch.float64, device="cuda")
                x = torch.zeros(s._level_shape(l), dtype=torch.float64, device="cuda")
                s.restrict_device(l, p, r, bc)
                s.prolong_device(l, p, e, x)
                outs.append((_host(bc), _host(x)))
            assert np.array_equal(outs[0][0], outs[1][0]), (l, p, "restriction")
            assert np.array_equal(outs[0][1], outs[1][1]), (l, p, "prolongation")
    sd.free()
    sh.free()
