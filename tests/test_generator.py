"""Checks of the seeded input generator (A = U diag(sigma) V^T, b = A x_* + r)."""
import math

import numpy as np
import pytest

from workloads import make_problem, sigma_geometric
from workloads.problems import draw_batch_shapes


@pytest.mark.parametrize("sigma", ["geometric", "half_ones"])
def test_singular_values_and_residual(sigma):
    m, n, kappa, rho = 1500, 40, 1e6, 1e-4
    p = make_problem(m, n, kappa, rho, seed=3, sigma=sigma)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    assert A.flags.f_contiguous and A.shape == (m, n)
    sv = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(sv, p.sigma, rtol=1e-9, atol=0)
    assert sv[0] / sv[-1] == pytest.approx(kappa, rel=1e-8)
    r = b - A @ xs
    assert np.linalg.norm(r) / (sv[0] * np.linalg.norm(xs)) == pytest.approx(rho, rel=1e-10)
    # residual orthogonal to range(A): A^T r = 0 up to rounding
    assert np.linalg.norm(A.T @ r) <= 1e-13 * sv[0] * (np.linalg.norm(r) + sv[0] * np.linalg.norm(xs))


def test_blockwise_basis_is_orthonormal():
    # above 200k rows U is assembled from independent orthonormal blocks
    p = make_problem(400_100, 8, 1e3, 1e-3, seed=4)
    A = p.numpy_A()
    sv = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(sv, sigma_geometric(8, 1e3), rtol=1e-10)


def test_seeded():
    a = make_problem(300, 10, 1e3, 1e-3, seed=5)
    b = make_problem(300, 10, 1e3, 1e-3, seed=5)
    c = make_problem(300, 10, 1e3, 1e-3, seed=6)
    assert np.array_equal(a.numpy_A(), b.numpy_A())
    assert not np.array_equal(a.numpy_A(), c.numpy_A())


def test_batch_shapes():
    shapes = draw_batch_shapes(512, seed=0)
    assert len(shapes) == 512
    for m, n, kappa, rho in shapes:
        assert 32 <= n <= 512 and 2000 <= m <= 50000 and m >= 20 * n
        assert 1e2 <= kappa <= 1e8 and 1e-10 <= rho <= 1e-2
    assert draw_batch_shapes(512, seed=0) == shapes
