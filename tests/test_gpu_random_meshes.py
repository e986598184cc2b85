"""Seeded random configurations against the oracle: 2D and 3D jittered meshes (some
graded, some non-cubic boxes), full, roller and symmetry boundary conditions, 1:100
random materials, random loads, FP64 or FP32 V-cycle, host or device setup, V-,
W-cycle or the additive form, Gauss-Seidel or Jacobi smoothing, default or
geometric-multigrid leaf capacity. Bars: the solution reaches rtol 1e-8 in the
true residual and is 0 at fixed components; FP64 within 1e-8 of the oracle's
solution (relative 2-norm) and +-1 iteration; FP32 V-cycle within 1e-6."""
import numpy as np
import pytest

from oracle import Oracle, OracleOptions
from workloads import box3d, small2d, small3d

torch = pytest.importorskip("torch")
from paper_2505_09064_amd import vasmg as V  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(i):
    rng = np.random.default_rng(5000 + i)
    dim = int(rng.integers(2, 4))
    nu = float(rng.uniform(0.25, 0.49))
    if dim == 2:
        n = int(rng.integers(5, 70))
        fix = str(rng.choice(["boundary", "x0", "symmetry"]))
        graded = bool(rng.random() < 0.3)
        m = small2d(n, seed=None if graded else int(rng.integers(0, 1000)), nu=nu, fix=fix, graded=graded)
    elif rng.random() < 0.25:
        nx, ny, nz = (int(v) for v in rng.integers(4, 14, size=3))
        m = box3d(nx, ny, nz, seed=int(rng.integers(0, 1000)), nu=nu)
    else:
        n = int(rng.integers(3, 17))
        fix = str(rng.choice(["x0", "symmetry", "roller_x1", "boundary"]))
        m = small3d(n, seed=int(rng.integers(0, 1000)), nu=nu, fix=fix)
    m.E = np.where(rng.random(m.elems.shape[0]) < 0.5, 1.0, 100.0)
    F = rng.normal(size=m.coords.shape) * (1 - m.fixed)
    prec = V.FP64 if rng.random() < 0.6 else V.FP32_PRECOND
    sdev = int(rng.random() < 0.5)
    cycle, smoother = "V", "colored"
    r = rng.random()
    if r < 0.15:
        cycle = "W"
    elif r < 0.25:
        cycle = "additive"
    elif r < 0.35:
        smoother = "jacobi"
    cap = (9 if dim == 2 else 27) if rng.random() < 0.15 else 0
    return m, F, prec, sdev, cycle, smoother, cap


@pytest.mark.parametrize("i", range(40))
def test_random_configuration_matches_oracle(i):
    m, F, prec, sdev, cycle, smoother, cap = _case(i)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed,
               OracleOptions(leaf_capacity=cap, cycle=cycle, smoother=smoother))
    xo, io = o.solve(F, 1e-8)
    opts = dict(precision=prec, setup_device=sdev, leaf_capacity=cap,
                cycle={"V": V.CYCLE_V, "W": V.CYCLE_W, "additive": V.CYCLE_ADDITIVE}[cycle],
                smoother=V.SMOOTHER_JACOBI if smoother == "jacobi" else V.SMOOTHER_GS)
    with V.Solver.from_mesh(m, **opts) as s:
        x, info = s.solve(F, 1e-8)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    case = (i, m.name, m.n_dofs, prec, sdev, cycle, smoother, cap)
    assert info["converged"] == 1 and info["rel_res_true"] < 1e-8, (case, info)
    assert np.all(x[m.fixed.astype(bool)] == 0.0), case
    if prec == V.FP64:
        assert abs(info["iterations"] - io["iterations"]) <= 1, (case, info["iterations"], io["iterations"])
        assert err <= 1e-8, (case, err)
    else:
        assert err <= 1e-6, (case, err)
