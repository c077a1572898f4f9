"""Pins of the oracle's operator, RHS and exact solvers."""
import numpy as np
import pytest
import scipy.linalg

from oracle import bspline, exact, operator as op, solvers
from workloads import normal_field

CASES = [
    ((8, 8, 8), 1, "periodic"), ((8, 8, 8), 3, "periodic"), ((7, 8, 9), 2, "dirichlet"),
    ((7, 5, 6), 1, "dirichlet"), ((8, 7, 8), 3, "dirichlet"), ((11, 12, 13), 5, "periodic"),
    ((11, 5, 7), 5, "dirichlet"), ((9, 10, 9), 4, "periodic"), ((6, 9, 7), 4, "dirichlet"),
]


@pytest.mark.parametrize("grid,n,bc", CASES)
def test_separable_apply_equals_dense_kronecker(grid, n, bc):
    h = (0.7, 1.3, 0.9)
    tau = 0.37
    u = normal_field(grid[::-1], 11)
    y = op.apply(u, n, h, tau, bc)
    A = op.dense_matrix(grid, n, h, tau, bc)
    assert np.allclose(y.ravel(), A @ u.ravel(), rtol=0, atol=1e-12 * np.abs(A).sum(1).max() * 4)
    # symmetric positive definite
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_periodic_constants_and_conservation(n):
    grid, h, tau = (12, 11, 13), (0.1, 0.2, 0.05), 0.03
    one = np.ones(grid[::-1])
    assert np.allclose(op.apply(one, n, h, tau, "periodic"), 1.0, atol=1e-13)
    u = normal_field(grid[::-1], 3)
    q = normal_field(grid[::-1], 4)
    u1 = exact.step(u, q, n, h, tau, "periodic")
    assert abs(u1.sum() - (u.sum() + tau * q.sum())) < 1e-10 * np.abs(u).sum()


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_polynomial_reproduction_interior(n):
    # interior rows reproduce quadratics: K k^2 = -2 and M k^2 = k^2 + (n+1)/6
    N = 40
    m, s = bspline.taps(n)
    k = np.arange(N, dtype=np.float64)
    M = op.matrix_1d(m, N, "dirichlet")
    K = op.matrix_1d(s, N, "dirichlet")
    inner = slice(n, N - n)
    assert np.allclose((K @ k ** 2)[inner], -2.0, atol=1e-10)
    assert np.allclose((M @ k ** 2)[inner], (k ** 2 + (n + 1) / 6.0)[inner], atol=1e-10)


@pytest.mark.parametrize("n", [1, 3, 5])
def test_dirichlet_is_zero_extension(n):
    # truncated bands == periodic bands on a grid padded with n zero planes on every side
    grid = (12, 13, 14)
    h, tau = (0.2, 0.3, 0.25), 0.11
    u = normal_field(grid[::-1], 21)
    up = np.zeros(tuple(N + 4 * n for N in grid[::-1]))
    sl = tuple(slice(2 * n, 2 * n + N) for N in grid[::-1])
    up[sl] = u
    y_per = op.apply(up, n, h, tau, "periodic")[sl]
    assert np.allclose(op.apply(u, n, h, tau, "dirichlet"), y_per, atol=1e-12)


def test_rhs_is_mass_of_shifted_state():
    grid = (9, 8, 10)
    u, q = normal_field(grid[::-1], 1), normal_field(grid[::-1], 2)
    n, tau = 3, 0.01
    A0 = op.dense_matrix(grid, n, (1, 1, 1), 1e-300, "dirichlet")  # tau -> 0 leaves the mass part
    b = op.rhs(u, q, n, tau, "dirichlet")
    assert np.allclose(b.ravel(), A0 @ (u + tau * q).ravel(), atol=1e-13)


@pytest.mark.parametrize("n", [1, 3, 5])
def test_fft_solve_matches_dense(n):
    grid = (11, 12, 11)
    h, tau = (0.3, 0.2, 0.25), 0.05
    b = normal_field(grid[::-1], 5)
    A = op.dense_matrix(grid, n, h, tau, "periodic")
    x = np.linalg.solve(A, b.ravel())
    assert np.allclose(exact.solve_periodic(b, n, h, tau).ravel(), x, atol=1e-11)


@pytest.mark.parametrize("n,grid", [(1, (6, 7, 8)), (3, (10, 9, 8)), (5, (12, 11, 12))])
def test_fast_diagonalisation_matches_cholesky(n, grid):
    h, tau = (0.1, 0.15, 0.12), 0.02
    b = normal_field(grid[::-1], 6)
    A = op.dense_matrix(grid, n, h, tau, "dirichlet")
    x = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b.ravel())
    assert np.allclose(exact.solve_dirichlet(b, n, h, tau).ravel(), x, atol=1e-10 * np.abs(x).max())


def test_fourier_mode_decay_closed_form():
    # 32^3 periodic cubic, h = 1/32, tau = 1e-3: a single Fourier mode decays by the factor
    # g = 1 / (1 + tau sum_d K(w_d) / (h^2 M(w_d))), with the symbols from Poisson summation
    n, N, tau = 3, 32, 1e-3
    h = (1.0 / N,) * 3
    x = np.arange(N)
    for (kx, ky, kz) in [(1, 0, 0), (1, 2, 3), (4, 4, 4), (16, 0, 5)]:
        w = [2 * np.pi * k / N for k in (kx, ky, kz)]
        mc, kc = bspline.symbol_closed_form(n, np.array(w))
        g = 1.0 / (1.0 + tau * N * N * np.sum(kc / mc))
        mode = np.cos(w[2] * x[:, None, None] + w[1] * x[None, :, None] + w[0] * x[None, None, :])
        u1 = exact.step(mode, None, n, h, tau, "periodic")
        assert np.allclose(u1, g * mode, atol=1e-13)
        # the same decay through the FFT-free route: A u1 == M u0 on the mode
        assert np.allclose(op.apply(g * mode, n, h, tau, "periodic"), op.rhs(mode, None, n, tau, "periodic"),
                           atol=1e-12)


def test_decay_values_of_the_32_cube():
    # re-derived reference values for the 32^3 periodic cubic step (tau = 1e-3, h = 1/32)
    n, N, tau = 3, 32, 1e-3
    g = exact.decay_factors((N, N, N), n, (1 / N,) * 3, tau)
    assert abs(g[0, 0, 1] - 0.962020935683587) < 1e-12
    assert abs(g[3, 2, 1] - 0.644040059555341) < 1e-12
    assert abs(g[4, 4, 4] - 0.345425098446613) < 1e-12


@pytest.mark.parametrize("bc,grid", [("periodic", (16, 12, 14)), ("dirichlet", (13, 12, 11))])
def test_cg_converges_to_exact_and_a_norm_decreases(bc, grid):
    n, h, tau = 3, (1 / 16, 1 / 12, 1 / 14), 2e-3
    u0 = normal_field(grid[::-1], 7)
    q = normal_field(grid[::-1], 8)
    b = op.rhs(u0, q, n, tau, bc)
    xs = exact.solve(b, n, h, tau, bc)
    A = lambda v: op.apply(v, n, h, tau, bc)
    errs = []
    for k in range(0, 12):
        x, it, _ = solvers.cg(A, b, u0, 0.0, 100, fixed_iters=k)
        e = x - xs
        errs.append(float(np.sum(e * A(e))))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    x, it, hist = solvers.cg(A, b, u0, 1e-12, 500)
    assert hist[-1] <= 1e-12
    kappa = exact.condition_number(grid, n, h, tau, bc)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 2 * kappa * 1e-12
    assert solvers.rel_residual(A, b, x) <= 2e-12


def test_cg_zero_rhs():
    A = lambda v: op.apply(v, 2, (1, 1, 1), 0.1, "periodic")
    x, it, hist = solvers.cg(A, np.zeros((5, 6, 7)), np.ones((5, 6, 7)), 1e-10, 10)
    assert it == 0 and np.all(x == 0)


def test_refinement_reaches_fp64_residual_with_fp32_inner():
    grid, n, bc, tau = (12, 12, 12), 3, "dirichlet", 1e-3
    h = (1 / 13,) * 3
    b = op.rhs(normal_field(grid[::-1], 9), None, n, tau, bc)
    A = lambda v: op.apply(v, n, h, tau, bc)
    A32 = lambda v: op.apply(v.astype(np.float32), n, h, tau, bc).astype(np.float32).astype(np.float64)

    def inner(r):
        d, _, _ = solvers.cg(A32, r.astype(np.float32).astype(np.float64), np.zeros_like(r), 1e-4, 200)
        return d.astype(np.float32).astype(np.float64)

    x, sweeps, rr = solvers.refine(A, b, np.zeros_like(b), 1e-12, inner)
    assert rr <= 1e-12 and 1 <= sweeps <= 6
    xs = exact.solve(b, n, h, tau, bc)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10


COND_CASES = [((6, 7, 8), 1, "periodic"), ((8, 7, 9), 3, "periodic"), ((11, 11, 12), 5, "periodic"),
              ((6, 7, 8), 1, "dirichlet"), ((9, 8, 7), 3, "dirichlet"), ((12, 11, 11), 5, "dirichlet")]


@pytest.mark.parametrize("grid,n,bc", COND_CASES)
def test_condition_number_against_dense_eigenvalues(grid, n, bc):
    # periodic grids: the symbol on the DFT grid gives the spectrum exactly; Dirichlet (truncated
    # bands): the eigenvalues lie inside the symbol's range, so the symbol's ratio bounds kappa
    h, tau = (0.11, 0.07, 0.13), 0.02
    lam = np.linalg.eigvalsh(op.dense_matrix(grid, n, h, tau, bc))
    kd = lam.max() / lam.min()
    ks = exact.condition_number(grid, n, h, tau, bc)
    if bc == "periodic":
        assert abs(ks - kd) <= 1e-9 * kd
    else:
        assert kd <= ks * (1 + 1e-12)
        # and the bound is not vacuous: the truncated spectrum fills most of the symbol's range
        assert kd >= 0.3 * ks
