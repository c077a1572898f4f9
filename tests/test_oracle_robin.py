"""Pins of the box-domain Robin / penalty oracle (oracle/robin.py) against what the B-spline
definitions fix: exact B-spline values, the Toeplitz taps inside the box, partition of unity,
linear and quadratic reproduction (closed-form integrals over the box), scipy's B-spline basis
integrated by adaptive quadrature, dense assembly, and the constant-coefficient operator on
fields that vanish near the boundary."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import bspline, operator as op, robin


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_float_bspline_equals_exact_values(p):
    xs = [Fraction(j, 7) for j in range(-25, 26)]
    got = robin.bspline_f(p, np.array([float(x) for x in xs]))
    ref = np.array([float(bspline.bspline(p, x)) for x in xs])
    assert np.allclose(got, ref, rtol=0, atol=1e-14)
    if p >= 1:
        d = robin.bspline_d(p, np.array([float(x) for x in xs]))
        dref = np.array([float(bspline.bspline(p - 1, x + Fraction(1, 2)) - bspline.bspline(p - 1, x - Fraction(1, 2)))
                         for x in xs])
        assert np.allclose(d, dref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_interior_rows_are_the_toeplitz_taps(n):
    N = 40
    M, K, E = robin.matrices_1d(N, n)
    m, s = bspline.taps(n)
    S = 2 * (n // 2) + 1  # rows that may differ at each end
    for i in range(S, N - S):
        for a in range(-n, n + 1):
            assert abs(M[i, i + a] - m[n + a]) < 1e-14
            assert abs(K[i, i + a] - s[n + a]) < 1e-13
        assert np.all(E[i] == 0.0)
    # outside the band the matrices vanish
    for i in range(N):
        for j in range(N):
            if abs(i - j) > n:
                assert M[i, j] == 0.0 and abs(K[i, j]) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("N", [2 * 5 + 3, 31])
def test_partition_of_unity_and_linear_reproduction(n, N):
    M, K, E = robin.matrices_1d(N, n)
    nc = robin.cells(N, n)
    k = robin.offsets(N, n).astype(np.float64)
    one = np.ones(N)
    # sum_k b(x - k) = 1 on the box: the integral of 1, no gradient, and one at both ends
    assert abs(one @ M @ one - nc) < 1e-12 * nc
    assert np.abs(K @ one).max() < 1e-13
    assert abs(one @ E @ one - 2.0) < 1e-14
    # sum_k k b(x - k) = x: int x^2 = nc^3/3, int 1 = nc, boundary values 0 and nc
    assert abs(k @ M @ k - nc ** 3 / 3) < 1e-12 * nc ** 3
    assert abs(k @ K @ k - nc) < 1e-12 * nc
    assert abs(k @ E @ k - nc ** 2) < 1e-12 * nc ** 2
    assert np.allclose(M, M.T, atol=1e-15) and np.allclose(K, K.T, atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_quadratic_reproduction(n):
    # sum_k k^2 b^n(x - k) = x^2 + (n+1)/12 for n >= 2 (variance of the (n+1)-fold box convolution)
    N = 27
    M, K, E = robin.matrices_1d(N, n)
    nc = robin.cells(N, n)
    k = robin.offsets(N, n).astype(np.float64)
    c = k * k
    C = (n + 1) / 12.0
    assert abs(c @ K @ c - 4.0 * nc ** 3 / 3.0) < 1e-11 * nc ** 3
    assert abs(c @ M @ c - (nc ** 5 / 5.0 + 2 * C * nc ** 3 / 3.0 + C * C * nc)) < 1e-11 * nc ** 5
    assert abs(c @ E @ c - (C * C + (nc * nc + C) ** 2)) < 1e-11 * nc ** 4


@pytest.mark.parametrize("n", [2, 3])
def test_matrices_equal_scipy_basis_integrated_by_quad(n):
    from scipy.integrate import quad
    from scipy.interpolate import BSpline
    N = 2 * n + 4
    M, K, E = robin.matrices_1d(N, n)
    nc = robin.cells(N, n)
    ks = robin.offsets(N, n)
    basis = [BSpline.basis_element(np.arange(n + 2) - (n + 1) / 2.0 + kk, extrapolate=False) for kk in ks]

    def f(b, x):
        v = b(x)
        return 0.0 if np.isnan(v) else float(v)

    def df(b, x):
        v = b.derivative()(x)
        return 0.0 if np.isnan(v) else float(v)

    pts = list(np.arange(0.0, nc + 0.01, 0.5))
    for i in range(N):
        for j in range(max(0, i - n), min(N, i + n + 1)):
            mij = quad(lambda x: f(basis[i], x) * f(basis[j], x), 0.0, nc, points=pts, limit=200)[0]
            kij = quad(lambda x: df(basis[i], x) * df(basis[j], x), 0.0, nc, points=pts, limit=200)[0]
            assert abs(M[i, j] - mij) < 1e-10
            assert abs(K[i, j] - kij) < 1e-10
        e_ref = [f(basis[i], 0.0) * f(basis[j], 0.0) + f(basis[i], nc) * f(basis[j], nc) for j in range(N)]
        assert np.allclose(E[i], e_ref, atol=1e-14)


def test_3d_apply_equals_dense_assembly_and_is_spd():
    grid, n, h, tau, gamma = (9, 8, 7), 3, (0.1, 0.12, 0.15), 2e-3, 0.05
    rng = np.random.default_rng(3)
    u = rng.standard_normal(grid[::-1])
    A = robin.dense_matrix(grid, n, h, tau, gamma)
    assert np.allclose(robin.apply(u, n, h, tau, gamma).ravel(), A @ u.ravel(), rtol=0, atol=1e-13)
    assert np.allclose(A, A.T, atol=1e-15)
    assert np.linalg.eigvalsh(A).min() > 0
    b = rng.standard_normal(grid[::-1])
    x = robin.solve(b, n, h, tau, gamma)
    assert np.linalg.norm(robin.apply(x, n, h, tau, gamma) - b) < 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_equals_truncated_operator_away_from_the_boundary(n):
    # on fields that vanish within 2 floor(n/2) + 1 rows of every face the Robin operator equals
    # the truncated-band constant-coefficient operator (the rows that differ see only zeros)
    grid, h, tau, gamma = (26, 22, 20), (0.04, 0.05, 0.06), 1e-3, 0.1
    S = 2 * (n // 2) + 1
    rng = np.random.default_rng(n)
    u = np.zeros(grid[::-1])
    u[S:-S, S:-S, S:-S] = rng.standard_normal((grid[2] - 2 * S, grid[1] - 2 * S, grid[0] - 2 * S))
    a = robin.apply(u, n, h, tau, gamma)
    b = op.apply(u, n, h, tau, "dirichlet")
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_penalty_limit_drives_the_boundary_trace_to_zero():
    # 1-D steady problem (K~ + E / (2 gamma)) c = M~ 1: the boundary value phi(0) = sum_k c_k b(-k)
    # falls like gamma as gamma -> 0 (weakly imposed Dirichlet condition)
    n, N = 3, 40
    M, K, E = robin.matrices_1d(N, n)
    k = robin.offsets(N, n)
    b0 = robin.bspline_f(n, 0.0 - k)
    trace = []
    for gamma in (1e-2, 1e-3, 1e-4):
        c = np.linalg.solve(K + E / (2 * gamma), M @ np.ones(N))
        trace.append(abs(b0 @ c))
    assert trace[1] < 0.2 * trace[0] and trace[2] < 0.2 * trace[1]
