"""Pins of the variable-coefficient oracle (oracle/varcoef.py): the three-index kernels against
scipy's B-spline basis integrated by adaptive quadrature and their symmetries, the partition-of-
unity reduction to the Galerkin taps, the constant-coefficient operator A, entry-by-entry dense
assembly, symmetry, linearity and positivity."""
import numpy as np
import pytest

from oracle import bspline, operator as op, varcoef
from workloads import normal_field


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_kernel_symmetries_and_partition_of_unity(n):
    F, W = varcoef.kernels_1d(n)
    m, s = bspline.taps(n)
    for p in range(-n, n + 1):
        for q in range(-n, n + 1):
            # int b(x-k) b(x-l) b(x-m): symmetric in k, l; swapping k and m maps (p, q) to (-p, q - p)
            assert abs(F[p + n, q + n] - F[q + n, p + n]) < 1e-15
            assert abs(W[p + n, q + n] - W[q + n, p + n]) < 1e-15
            if abs(q - p) <= n:
                assert abs(F[p + n, q + n] - F[-p + n, q - p + n]) < 1e-15
    # sum over the coefficient index m: the Galerkin taps (sum_m b_m = 1)
    for a in range(-n, n + 1):
        sf = sum(F[a + q + n, q + n] for q in range(-n, n + 1) if abs(a + q) <= n)
        sw = sum(W[a + q + n, q + n] for q in range(-n, n + 1) if abs(a + q) <= n)
        assert abs(sf - m[a + n]) < 1e-15
        assert abs(sw - s[a + n]) < 1e-14


@pytest.mark.parametrize("n", [2, 3])
def test_kernels_equal_scipy_basis_integrated_by_quad(n):
    from scipy.integrate import quad
    from scipy.interpolate import BSpline
    F, W = varcoef.kernels_1d(n)

    def el(k):
        return BSpline.basis_element(np.arange(n + 2) - (n + 1) / 2.0 + k, extrapolate=False)

    def ev(b, x, der=0):
        v = (b.derivative() if der else b)(x)
        return 0.0 if np.isnan(v) else float(v)

    b0 = el(0)
    pts = list(np.arange(-(n + 1) / 2.0, (n + 1) / 2.0 + 0.01, 0.5))
    for p in range(-n, n + 1):
        for q in range(-n, n + 1):
            bp, bq = el(p), el(q)
            lo, hi = -(n + 1) / 2.0, (n + 1) / 2.0
            f = quad(lambda x: ev(bp, x) * ev(bq, x) * ev(b0, x), lo, hi, points=pts, limit=200)[0]
            w = quad(lambda x: ev(bp, x, 1) * ev(bq, x, 1) * ev(b0, x), lo, hi, points=pts, limit=200)[0]
            assert abs(F[p + n, q + n] - f) < 1e-11
            assert abs(W[p + n, q + n] - w) < 1e-11


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_constant_coefficients_give_the_heat_operator(n, bc):
    grid, h, tau = (11, 9, 8), (0.1, 0.12, 0.15), 2e-3
    c = normal_field(grid[::-1], 4)
    one = np.ones(grid[::-1])
    got = varcoef.apply(c, tau * one, one, n, h, bc)
    ref = op.apply(c, n, h, tau, bc)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n,grid,bc", [(1, (4, 3, 3), "dirichlet"), (1, (4, 3, 3), "periodic"),
                                       (2, (5, 5, 5), "dirichlet"), (3, (4, 4, 4), "dirichlet")])
def test_apply_equals_entrywise_dense_assembly(n, grid, bc):
    h = (0.2, 0.25, 0.3)
    rng = np.random.default_rng(n)
    d = 0.01 + rng.random(grid[::-1])
    m = 0.5 + rng.random(grid[::-1])
    c = rng.standard_normal(grid[::-1])
    A = varcoef.dense_matrix(grid, d, m, n, h, bc)
    got = varcoef.apply(c, d, m, n, h, bc)
    assert np.abs(got.ravel() - A @ c.ravel()).max() < 1e-13 * np.abs(A @ c.ravel()).max()
    # a Galerkin matrix: symmetric; positive definite for positive coefficient fields
    assert np.allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0


def test_linear_in_the_coefficients_and_symmetric():
    grid, n, h, bc = (12, 10, 9), 3, (0.1, 0.1, 0.1), "dirichlet"
    rng = np.random.default_rng(7)
    c, v = rng.standard_normal(grid[::-1]), rng.standard_normal(grid[::-1])
    d1, d2 = rng.random(grid[::-1]), rng.random(grid[::-1])
    m1, m2 = rng.random(grid[::-1]), rng.random(grid[::-1])
    a = varcoef.apply(c, d1 + 2 * d2, m1 - m2, n, h, bc)
    b = varcoef.apply(c, d1, m1, n, h, bc) + 2 * varcoef.apply(c, d2, 0 * m2, n, h, bc) - varcoef.apply(c, 0 * d1, m2, n, h, bc)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()
    lhs = np.sum(v * varcoef.apply(c, d1, m1, n, h, bc))
    rhs = np.sum(c * varcoef.apply(v, d1, m1, n, h, bc))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
