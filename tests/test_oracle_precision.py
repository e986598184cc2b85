"""Pins of the oracle's FP32-emulation mode and of its flexible-beta PCG variant.

The mixed-precision mode keeps PCG (Section 2.2, Algorithm 2) in FP64 and runs
the V-cycle (Section 3, Algorithm 3 applied recursively) in single precision:
level matrices, prolongation weights and cycle vectors are float32, the
coarsest system is solved in FP64 and the result rounded back. These tests
fail if any of those pieces silently runs at the wrong precision:

  * dtypes of every stored operator, weight and smoother matrix;
  * with the fine level as the coarsest, the FP32 cycle returns exactly the
    float32 rounding of an FP64 direct solve of the float32-rounded input
    (an FP32 factorisation would differ in the last bits);
  * one FP32 Gauss-Seidel sweep equals a literal float32 point loop to within
    a few float32 ulps and differs from the FP64 sweep by more than FP64
    rounding could explain;
  * the FP32 cycle's distance from the FP64 cycle is of float32 size: above
    1e-9 (so it is not FP64) and below 1e-5 (so it is not broken).

The flexible beta r_new^T (z_new - z_old) / rho_old equals the printed
Fletcher-Reeves beta rho_new / rho_old whenever the preconditioner is a fixed
symmetric positive definite operator, because r_new^T z_old = 0 in exact
arithmetic; both variants must then produce the same iterates.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import Oracle, OracleOptions
from workloads import small2d, small3d

U32 = float(np.finfo(np.float32).eps) / 2      # unit roundoff of float32


def _mesh(dim):
    return small2d(9, seed=3) if dim == 2 else small3d(5, seed=4)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_mode_stores_single_precision(dim):
    m = _mesh(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    assert o.L >= 2
    vc = o.vcycle(precision="fp32")
    assert all(A.dtype == np.float32 for A in vc.A)
    assert all(P.dtype == np.float32 for P in vc.Pb + vc.PbT)
    for S in vc.smoothers:
        assert S.dtype == np.float32
        for comps in S.parts:
            for rows, Ar, aii in comps:
                assert Ar.dtype == np.float32 and aii.dtype == np.float32
    # the coarsest factor stays FP64
    assert o.coarsest.c[0].dtype == np.float64
    # vectors inside the cycle are single precision, FP64 at the PCG boundary
    r = np.random.default_rng(0).normal(size=o.A[0].shape[0])
    assert vc.apply(r).dtype == np.float32
    assert o.apply_precond(r, precision="fp32").dtype == np.float64
    # the FP64 cycle stays FP64
    vc64 = o.vcycle(precision="fp64")
    assert all(A.dtype == np.float64 for A in vc64.A)
    assert vc64.apply(r).dtype == np.float64


def test_fp32_coarsest_solve_is_fp64():
    # nearly incompressible, so an FP32 factorisation is visibly worse (kappa ~ 450)
    m = small2d(11, seed=1, nu=0.49)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(coarsest_max_dofs=10 ** 6))
    assert o.L == 0
    r = np.random.default_rng(1).normal(size=o.A[0].shape[0])
    z = o.apply_precond(r, precision="fp32")
    # the exact FP64 solve of the rounded input, then rounded: bit for bit
    r32 = r.astype(np.float32).astype(np.float64)
    ref = np.linalg.solve(o.A[0].toarray(), r32).astype(np.float32).astype(np.float64)
    assert np.abs(z - ref).max() <= 2 * U32 * np.abs(ref).max()
    # an FP32 factorisation is measurably different from that
    A32 = o.A[0].toarray().astype(np.float32)
    c32 = sla.cho_factor(A32, lower=True)
    z_bad = sla.cho_solve(c32, r.astype(np.float32)).astype(np.float64)
    assert np.abs(z_bad - ref).max() > 16 * U32 * np.abs(ref).max()
    # the gap the pin above tolerates is far below that difference
    assert np.abs(z - ref).max() < np.abs(z_bad - ref).max() / 4


def _literal_point_gs32(A, d, order, b, x):
    """Point Gauss-Seidel (Algorithm 1) with float32 scalars, visiting the
    vertices in `order` and their components ascending; each unknown is
    replaced by (b_i - sum_{j != i} a_ij x_j) / a_ii, summed left to right."""
    A = A.tocsr()
    x = [np.float32(v) for v in x]
    for v in order:
        for a in range(d):
            i = v * d + a
            s = np.float32(b[i])
            aii = np.float32(0)
            for p in range(A.indptr[i], A.indptr[i + 1]):
                j = A.indices[p]
                aij = np.float32(A.data[p])
                if j == i:
                    aii = aij
                else:
                    s = np.float32(s - np.float32(aij * x[j]))
            x[i] = np.float32(s / aii)
    return np.array(x, dtype=np.float64)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_sweep_is_single_precision_gauss_seidel(dim):
    m = _mesh(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    rng = np.random.default_rng(2)
    for l in range(min(2, o.L)):
        A = o.A[l]
        n = A.shape[0]
        b = rng.normal(size=n).astype(np.float32)
        x = rng.normal(size=n).astype(np.float32)
        S32 = o.gs(l, np.float32)
        S64 = o.gs(l, np.float64)
        y32 = S32.forward(b, x).astype(np.float64)
        y64 = S64.forward(b.astype(np.float64), x.astype(np.float64))
        nv = A.shape[0] // dim
        order = np.lexsort((np.arange(nv), o.cells[l], o.blocks[l],
                            o.block_colors[l][o.blocks[l]]))
        lit = _literal_point_gs32(A, dim, order, b, x)
        scale = np.abs(y64).max()
        # same arithmetic as a float32 loop up to summation order ...
        assert np.abs(y32 - lit).max() <= 64 * U32 * scale, l
        # ... and really float32: farther from the FP64 sweep than FP64 rounding
        gap = np.abs(y32 - y64).max() / scale
        assert 1e-9 < gap < 1e-5, (l, gap)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_cycle_distance_from_fp64_is_single_precision_sized(dim):
    m = _mesh(dim)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    r = np.random.default_rng(3).normal(size=o.A[0].shape[0])
    z64 = o.apply_precond(r, precision="fp64")
    z32 = o.apply_precond(r, precision="fp32")
    rel = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e-9 < rel < 1e-5, rel
    # and the mixed solve keeps the FP64 stopping rule and accuracy
    x64, i64 = o.solve(m.rhs[0], 1e-8)
    x32, i32 = o.solve(m.rhs[0], 1e-8, precision="fp32")
    assert i32["converged"] and i32["rel_res_true"] < 1e-8
    assert abs(i32["iterations"] - i64["iterations"]) <= 1
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-7


@pytest.mark.parametrize("dim", [2, 3])
def test_flexible_beta_equals_printed_beta_for_fixed_spd_preconditioner(dim):
    m = _mesh(dim)
    o_fr = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    o_fx = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed, OracleOptions(flexible=True))
    x1, i1 = o_fr.solve(m.rhs[0], 1e-10)
    x2, i2 = o_fx.solve(m.rhs[0], 1e-10)
    assert i1["converged"] and i2["converged"]
    assert i1["iterations"] == i2["iterations"]
    h1, h2 = np.array(i1["history"]), np.array(i2["history"])
    assert np.abs(h1 - h2).max() <= 1e-6 * h1.max()
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)


def test_flexible_beta_branch_is_taken_under_a_varying_preconditioner():
    """With a preconditioner that changes from one application to the next
    (alternately the V-cycle and a point-Jacobi step), r_new^T z_old no longer
    vanishes: the two beta formulas must then give different iterates, and the
    flexible one must still converge."""
    from oracle.pcg import pcg
    m = small3d(5, seed=4)
    o = Oracle(m.coords, m.elems, m.E, m.nu, m.fixed)
    A = o.A[0]
    F = o.to_free(m.rhs[0])
    dinv = 1.0 / A.diagonal()
    vc = o.vcycle()

    def varying():
        k = [0]

        def M(r):
            k[0] += 1
            return vc.apply(r) if k[0] % 2 else dinv * r
        return M

    _, i_fr = pcg(A, F, varying(), 1e-8, 500, None, False)
    _, i_fx = pcg(A, F, varying(), 1e-8, 500, None, True)
    assert i_fx["converged"]
    n = min(len(i_fr["history"]), len(i_fx["history"]))
    h1, h2 = np.array(i_fr["history"][:n]), np.array(i_fx["history"][:n])
    assert np.abs(h1[3:] - h2[3:]).max() > 1e-3 * np.abs(h1[3:]).max()
