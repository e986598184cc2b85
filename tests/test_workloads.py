"""Input generators: the batched Fourier load generator equals the per-case
quadrature definition, and integrates polynomials exactly (degree-2 rule)."""
import numpy as np

from workloads import fourier_body_force, load_fourier_tet, load_function_tet, small3d


def test_batched_fourier_loads_equal_the_per_case_rule():
    m = small3d(9, seed=3, fix="x0")
    A = [load_function_tet(m.coords, m.elems, fourier_body_force(r)) for r in range(5)]
    B = load_fourier_tet(m.coords, m.elems, 5, chunk=700)      # several ragged chunks
    for a, b in zip(A, B):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_quadrature_integrates_quadratics_exactly():
    # sum_v F_v = integral of f over the domain (partition of unity); f = x*y in each component
    m = small3d(7, seed=2, fix="none")
    F = load_function_tet(m.coords, m.elems, lambda x, y, z: np.stack([x * y, y * z, x * x], 1))
    assert np.allclose(F.sum(axis=0), [0.25, 0.25, 1.0 / 3.0], rtol=0, atol=1e-13)
