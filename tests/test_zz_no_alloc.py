"""The no-allocation host-pointer solve (vasmg_solve_noalloc) against the
allocating one (vasmg_solve) through the C ABI: identical solutions and
reports on two calls in a row, the second with a smaller input (another,
smaller mesh and fewer right-hand sides) that reuses the same fixed staging
array; a request beyond the array is refused before anything is copied."""
import numpy as np
import pytest

from workloads import small2d, small3d

torch = pytest.importorskip("torch")
from paper_2505_09064_amd import vasmg as V  # noqa: E402

pytestmark = pytest.mark.gpu


def _same(a, b):
    xa, ia = a
    xb, ib = b
    assert np.array_equal(xa, xb), np.abs(xa - xb).max()
    ia = ia if isinstance(ia, list) else [ia]
    ib = ib if isinstance(ib, list) else [ib]
    for p, q in zip(ia, ib):
        for k in ("iterations", "converged", "rel_res", "rel_res_true", "status"):
            assert p[k] == q[k], (k, p[k], q[k])


@pytest.mark.parametrize("prec", [V.FP64, V.FP32_PRECOND])
def test_noalloc_solve_equals_allocating_solve(prec):
    big = small3d(9, seed=5)
    small = small2d(11, seed=3)
    sb = V.Solver.from_mesh(big, precision=prec)
    ss = V.Solver.from_mesh(small, precision=prec)
    # first call: 3 right-hand sides with initial guesses on the larger mesh
    F = np.stack([big.rhs[0], -2.0 * big.rhs[0], big.rhs[0] + 0.25])
    x0 = 1e-3 * np.random.default_rng(0).normal(size=F.shape)
    x0[:, big.fixed.any(axis=1)] = 0.0
    _same(sb.solve_noalloc(F, 1e-8, x0=x0), sb.solve(F, 1e-8, x0=x0))
    # second call: one right-hand side, no initial guess, on the smaller mesh
    _same(ss.solve_noalloc(small.rhs[0], 1e-8), ss.solve(small.rhs[0], 1e-8))
    # and the larger one again, after the smaller call left its data behind
    _same(sb.solve_noalloc(F[1], 1e-6), sb.solve(F[1], 1e-6))
    # beyond the fixed array: refused with EINVAL, x untouched
    n = (64 << 20) // (big.n_vertices * 3 * 8 * 2) + 1
    Fbig = np.zeros((n, big.n_vertices, 3))
    with pytest.raises(V.VasmgError) as e:
        sb.solve_noalloc(Fbig, 1e-6)
    assert e.value.status == V.EINVAL and "staging" in str(e.value)
    sb.free()
    ss.free()
