"""Centred uniform B-splines and the 1-D Galerkin taps (oracle; test infrastructure only).

Paper: Sec. 2.3 "B-spline Spaces", Table 1 (tblBsplines):
  * support (-(p+1)/2, (p+1)/2), symmetric (rows "sign and support", "structure");
  * derivative rule  d/dx b^p(x) = b^{p-1}(x+1/2) - b^{p-1}(x-1/2)   (row "derivative");
  * b^p is the (p+1)-fold convolution of b^0                           (row "convolution");
  * scalar product   int b^m(x-k) b^n(x-l) dx = b^{m+n+1}(k-l)          (row "scalar product").

With m = n the scalar-product row gives the mass taps m_k = b^{2n+1}(k).  Differentiating
that identity once in k and once in l gives int b^n'(x-k) b^n'(x-l) dx = -(b^{2n+1})''(k-l),
so the stiffness taps are s_k = -(b^{2n+1})''(k); applying the derivative row twice writes
(b^p)'' as the second difference b^{p-2}(x+1) - 2 b^{p-2}(x) + b^{p-2}(x-1).

The closed form used for b^p is the truncated-power expansion of the (p+1)-fold
convolution of the unit box (a textbook identity):
  b^p(x) = 1/p! * sum_{j=0}^{p+1} (-1)^j C(p+1, j) (x + (p+1)/2 - j)_+^p .
"""
from fractions import Fraction
from math import comb, factorial, pi

import numpy as np


def bspline(p, x):
    """Exact value of the centred B-spline b^p at a rational point x (Fraction in, Fraction out)."""
    if p < 0:
        raise ValueError("degree must be >= 0")
    x = Fraction(x)
    half = Fraction(p + 1, 2)
    if not (-half < x < half):
        return Fraction(0)
    acc = Fraction(0)
    for j in range(p + 2):
        t = x + half - j
        if t > 0:
            acc += (-1) ** j * comb(p + 1, j) * t ** p
    return acc / factorial(p)


def bspline_dd(p, x):
    """Exact second derivative of b^p at x via the derivative row of Table 1 applied twice (p >= 2)."""
    if p < 2:
        raise ValueError("second derivative needs p >= 2")
    x = Fraction(x)
    return bspline(p - 2, x + 1) - 2 * bspline(p - 2, x) + bspline(p - 2, x - 1)


def taps_exact(n):
    """Exact one-sided Galerkin taps for basis degree n.

    Returns (m, s): lists of Fractions indexed k = 0..n, the taps being symmetric in k.
      m_k = b^{2n+1}(k)        (mass; Table 1 scalar-product row with m = n)
      s_k = -(b^{2n+1})''(k)   (stiffness; same identity differentiated in k and l)
    """
    if not (1 <= n <= 5):
        raise ValueError("degree n must be in 1..5")
    p = 2 * n + 1
    m = [bspline(p, k) for k in range(n + 1)]
    s = [-bspline_dd(p, k) for k in range(n + 1)]
    return m, s


def taps(n):
    """FP64 full (two-sided) taps, index j = 0..2n  <->  offset k = j - n."""
    m, s = taps_exact(n)
    mf = np.array([float(m[abs(k)]) for k in range(-n, n + 1)], dtype=np.float64)
    sf = np.array([float(s[abs(k)]) for k in range(-n, n + 1)], dtype=np.float64)
    return mf, sf


def symbol_from_taps(t, omega):
    """Fourier symbol of a symmetric filter t (two-sided, length 2n+1) at angular frequency omega."""
    n = (len(t) - 1) // 2
    omega = np.asarray(omega, dtype=np.float64)
    acc = np.full(omega.shape, t[n], dtype=np.float64)
    for k in range(1, n + 1):
        acc = acc + 2.0 * t[n + k] * np.cos(k * omega)
    return acc


def symbol_closed_form(n, omega, terms=200):
    """Mass and stiffness symbols of degree-n B-splines by Poisson summation.

    The Fourier transform of b^n is sinc^{n+1}(xi/2) (sinc(x) = sin x / x), so sampling
    b^{2n+1} at the integers has the DTFT sum_j sinc^{2n+2}((omega + 2 pi j)/2), and the
    sampled negated second derivative has sum_j (omega + 2 pi j)^2 sinc^{2n+2}(...).
    Since sin^{2n+2}(omega/2 + pi j) = sin^{2n+2}(omega/2), the terms with |j| > J sum in closed
    form with the Hurwitz zeta function; the result is exact up to rounding.
    This is independent of the truncated-power formula and of the taps.
    """
    from scipy.special import zeta

    omega = np.asarray(omega, dtype=np.float64)
    j = np.arange(-terms, terms + 1, dtype=np.float64)
    xi = omega[..., None] + 2.0 * pi * j
    half = xi / 2.0
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(half == 0.0, 1.0, np.sin(half) / np.where(half == 0.0, 1.0, half))
    w = sinc ** (2 * n + 2)
    mass = w.sum(axis=-1)
    stiff = (xi * xi * w).sum(axis=-1)
    # tails: (2 sin(omega/2))^{2n+2} * sum_{|j|>J} (omega + 2 pi j)^{-e},  e = 2n+2 (mass), 2n (stiffness)
    amp = (2.0 * np.sin(omega / 2.0)) ** (2 * n + 2)
    a = omega / (2.0 * pi)
    for e, which in ((2 * n + 2, 0), (2 * n, 1)):
        tail = (zeta(e, terms + 1 + a) + zeta(e, terms + 1 - a)) / (2.0 * pi) ** e
        if which == 0:
            mass = mass + amp * tail
        else:
            stiff = stiff + amp * tail
    return mass, stiff
