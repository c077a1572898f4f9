"""Oracle coarse-grid guess against what fixes it: the two-scale relation on exact B-spline values,
adjointness of restriction and prolongation, and the Galerkin identity P^T A P / 8 = A(2h) on a
periodic grid (dense assembly)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import coarse, operator as op, solvers
from oracle.bspline import bspline
import workloads


@pytest.mark.parametrize("n", [1, 3, 5])
def test_two_scale_relation_on_exact_values(n):
    # a periodic coarse spline sum_j C_j beta^n(y/2 - j) equals the fine spline of prolong(C)
    N, Nc = 24, 12
    rng = np.random.default_rng(n)
    C = rng.standard_normal(Nc)
    c = coarse.prolong_1d(C[None, None, :], N, 2, n, "periodic")[0, 0]
    for y in [Fraction(k, 3) for k in range(0, 3 * N, 5)]:
        fine = sum(c[i] * float(bspline(n, y - i - m * N)) for i in range(N) for m in (-1, 0, 1))
        crs = sum(C[j] * float(bspline(n, y / 2 - j - m * Nc)) for j in range(Nc) for m in (-1, 0, 1))
        assert abs(fine - crs) <= 1e-13


def test_weights_sum_and_even_degrees_rejected():
    for n in (1, 3, 5):
        assert abs(sum(coarse.weights(n).values()) - 2.0) <= 1e-15
    with pytest.raises(ValueError):
        coarse.weights(2)


@pytest.mark.parametrize("bc,grid", [("periodic", (16, 12, 14)), ("dirichlet", (17, 12, 15))])
def test_restrict_is_adjoint_of_prolong(bc, grid):
    rng = np.random.default_rng(1)
    gc = coarse.coarse_grid(grid, bc)
    C = rng.standard_normal(gc[::-1])
    f = rng.standard_normal(grid[::-1])
    lhs = np.sum(coarse.prolong(C, grid, 3, bc) * f)
    rhs = np.sum(C * coarse.restrict(f, grid, 3, bc))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_galerkin_projection_equals_coarse_operator_periodic():
    n, grid, tau = 3, (14, 14, 14), 3e-3
    h = (1 / 14, 1 / 14, 1 / 14)
    gc = coarse.coarse_grid(grid, "periodic")
    A = op.dense_matrix(grid, n, h, tau, "periodic")
    Nc = gc[0] * gc[1] * gc[2]
    P = np.zeros((grid[0] * grid[1] * grid[2], Nc))
    for j in range(Nc):
        e = np.zeros(Nc)
        e[j] = 1.0
        P[:, j] = coarse.prolong(e.reshape(gc[::-1]), grid, n, "periodic").ravel()
    Ac = op.dense_matrix(gc, n, tuple(2 * v for v in h), tau, "periodic")
    assert np.allclose(P.T @ A @ P / 8.0, Ac, rtol=0, atol=1e-12 * np.abs(Ac).max())


def test_coarse_guess_reduces_residual_and_iterations():
    n, N = 3, 31
    grid, h = (N,) * 3, (1 / (N + 1),) * 3
    tau = 8.6 * h[0] ** 2
    u = workloads.gaussian_sum(grid, "dirichlet", h, workloads.gaussian_params(3, 16, 0.02, 0.1, 1.0, 0.1, 0.9))
    b = op.rhs(u, None, n, tau, "dirichlet")
    A = lambda v: op.apply(v, n, h, tau, "dirichlet")
    x0, it_c = coarse.guess(u, b, n, h, tau, "dirichlet", 1e-2)
    assert it_c >= 1
    assert solvers.rel_residual(A, b, x0) <= 0.2 * solvers.rel_residual(A, b, u)
    _, it_plain, _ = solvers.cg(A, b, u, 1e-8, 500)
    _, it_coarse, _ = solvers.cg(A, b, x0, 1e-8, 500)
    assert it_coarse < it_plain
