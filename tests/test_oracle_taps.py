"""Pins of the oracle's B-spline taps and symbols against facts fixed outside the oracle."""
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy.interpolate import BSpline

from oracle import bspline
from oracle.operator import DIRICHLET, matrix_1d


def test_linear_is_textbook_fem():
    # n = 1: the linear B-spline Galerkin matrices are the textbook linear-FEM ones,
    # mass h [1/6, 2/3, 1/6] and stiffness h^-1 [-1, 2, -1].
    m, s = bspline.taps_exact(1)
    assert m == [Fraction(2, 3), Fraction(1, 6)]
    assert s == [Fraction(2), Fraction(-1)]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_moments(n):
    # partition of unity: mass rows sum to 1; constants are in the stiffness kernel;
    # the variance of b^{2n+1} is (2n+2)/12; K reproduces -(x^2)'' = -2 exactly.
    m, s = bspline.taps_exact(n)
    two = lambda t: [t[abs(k)] for k in range(-n, n + 1)]
    M, S = two(m), two(s)
    ks = range(-n, n + 1)
    assert sum(M) == 1
    assert sum(S) == 0
    assert sum(mk * k * k for mk, k in zip(M, ks)) == Fraction(n + 1, 6)
    assert sum(sk * k * k for sk, k in zip(S, ks)) == -2
    assert all(mk > 0 for mk in M)


def _quad_products(n, k, deriv):
    """int B(x) B(x - k) dx (or with first derivatives) with scipy's B-spline and exact Gauss."""
    knots = np.arange(n + 2, dtype=np.float64) - (n + 1) / 2.0
    b0 = BSpline.basis_element(knots, extrapolate=False)
    if deriv:
        b0 = b0.derivative()
    xg, wg = leggauss(n + 2)  # exact for piecewise polynomials of degree <= 2n+3
    lo, hi = -(n + 1) / 2.0, (n + 1) / 2.0 + k
    total = 0.0
    for j in range(int(round(hi - lo))):  # knot intervals [lo + j, lo + j + 1] of both factors
        x = lo + j + 0.5 + 0.5 * xg
        f = np.nan_to_num(b0(x)) * np.nan_to_num(b0(x - k))
        total += 0.5 * np.sum(wg * f)
    return total


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_taps_match_library_quadrature(n):
    # Galerkin entries integrated directly with scipy's B-spline basis element (a library
    # evaluation of the B-spline, independent of the truncated-power formula).
    m, s = bspline.taps(n)
    for k in range(0, n + 1):
        assert abs(_quad_products(n, k, False) - m[n + k]) < 1e-13
        assert abs(_quad_products(n, k, True) - s[n + k]) < 1e-12


def test_appendix_values_n3():
    m, s = bspline.taps_exact(3)
    assert m == [Fraction(151, 315), Fraction(397, 1680), Fraction(1, 42), Fraction(1, 5040)]
    assert s == [Fraction(2, 3), Fraction(-1, 8), Fraction(-1, 5), Fraction(-1, 120)]


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_symbol_matches_poisson_sum(n):
    m, s = bspline.taps(n)
    w = np.linspace(0.0, np.pi, 17)
    mc, kc = bspline.symbol_closed_form(n, w)
    assert np.allclose(bspline.symbol_from_taps(m, w), mc, rtol=0, atol=1e-12)
    assert np.allclose(bspline.symbol_from_taps(s, w), kc, rtol=0, atol=1e-12)


def test_symbol_linear_closed_form():
    m, s = bspline.taps(1)
    w = np.linspace(0, np.pi, 9)
    assert np.allclose(bspline.symbol_from_taps(m, w), (2 + np.cos(w)) / 3, atol=1e-15)
    assert np.allclose(bspline.symbol_from_taps(s, w), 2 - 2 * np.cos(w), atol=1e-15)


def _load_table():
    rows = []
    with open(__file__.replace("test_oracle_taps.py", "golden/table_flop1d_bspline.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def test_table_flop1d_truncated_bands():
    # The paper's operation counts for the 1-D B-spline matvec pin the truncated band structure
    # of the oracle's Dirichlet matrices (boundary rows have fewer nonzeros).
    for row in _load_table():
        h, counts = row[0], row[1:]
        for n, expected in zip(range(1, 6), counts):
            Nb = int(round(50 / h)) + 1 + 2 * (n // 2)
            m, s = bspline.taps(n)
            A = matrix_1d(m, Nb, DIRICHLET) + matrix_1d(s, Nb, DIRICHLET)
            nnz = np.count_nonzero(A, axis=1)
            assert int(np.sum(2 * nnz - 1)) == int(expected), (h, n)
