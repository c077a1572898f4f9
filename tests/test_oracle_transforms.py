"""Oracle B-spline transforms against what fixes them: scipy's own B-spline basis and its recursive
prefilter (the paper's direct-transform method, periodic grids), dense Kronecker assembly, partition
of unity and linear reproduction."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import transforms as tr
from oracle.operator import matrix_1d

scipy_interp = pytest.importorskip("scipy.interpolate")
scipy_ndimage = pytest.importorskip("scipy.ndimage")


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_eval_taps_are_basis_values_with_unit_sum(n):
    t = tr.eval_taps_exact(n)
    W = tr.eval_halfwidth(n)
    assert t[0] + 2 * sum(t[1:]) == 1
    # scipy's B-spline basis element on the uniform knots -(n+1)/2 .. (n+1)/2
    knots = np.arange(n + 2) - (n + 1) / 2
    b = scipy_interp.BSpline.basis_element(knots, extrapolate=False)
    for k in range(W + 1):
        assert abs(float(t[k]) - float(b(k))) <= 1e-15
    if n == 3:
        assert t == [Fraction(2, 3), Fraction(1, 6)]


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("n", [2, 3, 5])
def test_evaluate_and_interpolate_match_dense_kronecker(n, bc):
    grid = (7, 6, 5) if bc == "dirichlet" else (7, 6, 5)
    rng = np.random.default_rng(n)
    c = rng.standard_normal(grid[::-1])
    t = tr.eval_taps(n)
    Bx, By, Bz = (matrix_1d(t, N, bc) for N in grid)
    E = np.kron(Bz, np.kron(By, Bx))  # index z * Ny * Nx + y * Nx + x
    s = tr.evaluate(c, n, bc)
    assert np.allclose(s.ravel(), E @ c.ravel(), rtol=0, atol=1e-14)
    c2 = tr.interpolate(s, n, bc)
    assert np.allclose(c2.ravel(), np.linalg.solve(E, s.ravel()), rtol=0, atol=1e-12)
    assert np.allclose(c2, c, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_periodic_interpolate_equals_scipy_recursive_prefilter(n):
    # scipy.ndimage's spline prefilter is the recursive filtering of Unser's direct transform;
    # with mode 'grid-wrap' it solves the same circulant systems
    rng = np.random.default_rng(10 + n)
    s = rng.standard_normal((9, 12, 16))
    ref = scipy_ndimage.spline_filter(s, order=n, mode="grid-wrap")
    assert np.allclose(tr.interpolate(s, n, "periodic"), ref, rtol=0, atol=1e-10)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_linear_reproduction_and_constants(n):
    W = tr.eval_halfwidth(n)
    z, y, x = np.meshgrid(np.arange(8), np.arange(9), np.arange(10), indexing="ij")
    c = 0.5 + 2.0 * x - 1.5 * y + 0.25 * z
    s = tr.evaluate(c, n, "dirichlet")
    inner = (slice(W, -W),) * 3
    assert np.allclose(s[inner], c[inner], rtol=0, atol=1e-12)
    assert np.allclose(tr.evaluate(np.ones((8, 9, 10)), n, "periodic"), 1.0, rtol=0, atol=1e-15)
