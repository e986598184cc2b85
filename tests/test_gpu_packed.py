"""Packed solves (vasmg_pack, vasmg_solve_packed*): several small problems in
one block-diagonal hierarchy, each with its own PCG recurrence.

Bars: each part's result against the oracle's solve of that part (FP64: 1e-8
relative solution error and +-1 iteration; FP32 V-cycle: +-1 iteration of the
oracle's FP32 mode and 1e-5 of its FP64 solution), and against the same part
solved alone on the GPU (FP64: 1e-10 relative, +-1 iteration: the dot products
sum in another order). The packed V-cycle restricted to a part equals the
part's own V-cycle to rounding (1e-12 FP64), also for parts shallower than the
pack (their repeated coarsest levels end in an exact coarse solve)."""
import numpy as np
import pytest

from oracle import Oracle
from workloads import small2d, small3d

torch = pytest.importorskip("torch")
from paper_2505_09064_amd import vasmg as V  # noqa: E402

pytestmark = pytest.mark.gpu

PACKS = {
    "2d": lambda: [small2d(5, seed=1), small2d(17, seed=2, fix="symmetry"), small2d(9, seed=3),
                   small2d(17, seed=None, graded=True, nu=0.49), small2d(13, seed=4, fix="x0")],
    "3d": lambda: [small3d(5, seed=1), small3d(7, seed=2, fix="roller_x1"), small3d(4, seed=3),
                   small3d(9, seed=5)],
}


def _loads(meshes, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for m in meshes:
        m.E = np.where(rng.random(m.elems.shape[0]) < 0.5, 1.0, 100.0)
        out.append(rng.normal(size=m.coords.shape) * (1 - m.fixed))
    return out


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("name", list(PACKS))
@pytest.mark.parametrize("prec", [V.FP64, V.FP32_PRECOND])
def test_packed_solve_matches_oracle_and_alone(name, prec):
    meshes = PACKS[name]()
    F = _loads(meshes)
    parts = [V.Solver.from_mesh(m, host_only=1, precision=prec) for m in meshes]
    pk = V.PackedSolver(parts)
    X, infos = pk.solve_packed(F, 1e-6)
    for i, (m, f, x, info) in enumerate(zip(meshes, F, X, infos)):
        assert info["converged"] == 1 and info["rel_res_true"] < 1e-6, (i, info)
        o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
        xo, io = o.solve(f, 1e-6)
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        if prec == V.FP64:
            assert abs(info["iterations"] - io["iterations"]) <= 1, (i, info["iterations"], io)
            assert err <= 1e-8, (i, err)
        else:
            _, io32 = o.solve(f, 1e-6, precision="fp32")
            assert abs(info["iterations"] - io32["iterations"]) <= 1, (i, info["iterations"], io32)
            assert err <= 1e-5, (i, err)
        with V.Solver.from_mesh(m, precision=prec, autotune=0) as s:
            xa, ia = s.solve(f, 1e-6)
        assert abs(info["iterations"] - ia["iterations"]) <= 1, (i, info["iterations"], ia)
        if prec == V.FP64:
            assert np.linalg.norm(x - xa) / np.linalg.norm(xa) <= 1e-10, i
        assert np.all(x[m.fixed.astype(bool)] == 0.0)
    pk.free()


@pytest.mark.parametrize("name", list(PACKS))
def test_packed_vcycle_is_each_parts_vcycle(name):
    """z = B r of the packed handle, restricted to a part, is the part's own
    z = B r (FP64), including parts that end above the pack's coarsest level."""
    meshes = PACKS[name]()
    _loads(meshes)
    parts = [V.Solver.from_mesh(m, host_only=1) for m in meshes]
    depth = [p.hierarchy_info()[0] for p in parts]
    assert len(set(depth)) > 1
    pk = V.PackedSolver(parts)
    rng = np.random.default_rng(7)
    rs = [rng.normal(size=(p.hierarchy_info()[1] // m.dim, m.dim)) for p, m in zip(parts, meshes)]
    # the V-cycle works on the fine level's canonical order (free vertices of
    # each part, one part after the other)
    r = _dev(np.concatenate(rs))
    z = torch.zeros_like(r)
    V._check(V.lib().vasmg_apply_precond_device(pk.handle, V._ptr(r), V._ptr(z), None))
    torch.cuda.synchronize()
    zp = z.cpu().numpy()
    off = 0
    for m, ri in zip(meshes, rs):
        with V.Solver.from_mesh(m, autotune=0) as s:
            ra, za = _dev(ri), torch.zeros_like(_dev(ri))
            V._check(V.lib().vasmg_apply_precond_device(s.handle, V._ptr(ra), V._ptr(za), None))
            torch.cuda.synchronize()
            zi = za.cpu().numpy()
        n = ri.shape[0]
        assert np.abs(zp[off:off + n] - zi).max() <= 1e-12 * np.abs(zi).max()
        off += n
    pk.free()


def test_packed_parts_with_nothing_to_solve_and_device_entry():
    """A part with a zero load finishes at once (0 iterations, x = 0) while the
    others iterate; the device entry point gives the host entry point's result
    bit for bit; the ordinary solve calls refuse a packed handle."""
    meshes = [small2d(9, seed=1), small2d(13, seed=2), small2d(5, seed=3)]
    F = _loads(meshes)
    F[1] = np.zeros_like(F[1])
    parts = [V.Solver.from_mesh(m, host_only=1) for m in meshes]
    pk = V.PackedSolver(parts)
    X, infos = pk.solve_packed(F, 1e-8)
    assert infos[1]["iterations"] == 0 and infos[1]["converged"] == 1
    assert np.all(X[1] == 0.0)
    assert infos[0]["iterations"] > 0 and infos[2]["iterations"] > 0
    d_rhs = _dev(np.concatenate(F))
    d_x = torch.zeros_like(d_rhs)
    inf2 = pk.solve_packed_device(d_rhs, d_x, 1e-8)
    torch.cuda.synchronize()
    assert np.array_equal(d_x.cpu().numpy(), np.concatenate(X))
    assert [i["iterations"] for i in inf2] == [i["iterations"] for i in infos]
    with pytest.raises(V.VasmgError) as ei:
        pk.solve_device(d_rhs, d_x, 1e-8)
    assert ei.value.status == V.EINVAL
    pk.free()
