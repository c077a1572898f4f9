"""Direct and indirect B-spline transforms (oracle; test infrastructure only).

Table 1, interpolation row, and Sec. 2.3 (the signal-processing framework of Fig.
figBspnSignProc): the indirect transform evaluates a spline at the grid nodes,
s_k = sum_l c_l b^n(k - l), a convolution with the sampled B-spline b^n_k = beta^n(k); the direct
transform inverts it, c = (b^n)^{-1} * s.  Sec. 2.5 (method overview) places them before the solve
(source and coefficients into B-spline space) and after it (solution back to samples).

In 3-D both act as tensor products over the three axes.  Finite grids: periodic = circular
convolution; Dirichlet = coefficients outside the index box are zero (the truncated band of the
operator's reading), so the direct transform is the exact solution of the banded system.  Arrays
are numpy [z, y, x].
"""
from fractions import Fraction

import numpy as np
import scipy.linalg

from .bspline import bspline
from .operator import DIRICHLET, PERIODIC, filter_1d


def eval_halfwidth(n):
    """Largest |k| with beta^n(k) != 0: floor(n / 2)."""
    return n // 2


def eval_taps_exact(n):
    """b^n_k = beta^n(k) for k = 0..floor(n/2) as exact Fractions (symmetric in k)."""
    if not (2 <= n <= 5):
        raise ValueError("transform degree must be in 2..5")
    return [bspline(n, Fraction(k)) for k in range(eval_halfwidth(n) + 1)]


def eval_taps(n):
    """FP64 two-sided taps, index j = 0..2W <-> offset k = j - W."""
    t = eval_taps_exact(n)
    W = eval_halfwidth(n)
    return np.array([float(t[abs(k)]) for k in range(-W, W + 1)], dtype=np.float64)


def evaluate(c, n, bc):
    """Indirect transform: s = (Bx (x) By (x) Bz) c with the sampled B-spline along each axis."""
    t = eval_taps(n)
    c = np.asarray(c, dtype=np.float64)
    return filter_1d(filter_1d(filter_1d(c, t, "x", bc), t, "y", bc), t, "z", bc)


def _solve_axis(s, t, axis, bc):
    """Solve the 1-D system B c = s along one axis of a 3-D array (B banded or circulant)."""
    W = (len(t) - 1) // 2
    s = np.moveaxis(s, axis, -1)
    N = s.shape[-1]
    rhs = s.reshape(-1, N).T  # [N, lines]
    if bc == PERIODIC:
        col = np.zeros(N)
        for k in range(-W, W + 1):
            col[k % N] += t[W + k]  # first column of the circulant: B[i, 0] = t_{-i}
        out = scipy.linalg.solve_circulant(col, rhs)
    else:
        ab = np.zeros((2 * W + 1, N))
        for k in range(-W, W + 1):
            # banded storage: ab[W + i - j, j] = B[i, j] = t_{j - i}
            d = -k  # i - j
            if d >= 0:
                ab[W + d, : N - d] = t[W + k]
            else:
                ab[W + d, -d:] = t[W + k]
        out = scipy.linalg.solve_banded((W, W), ab, rhs)
    return np.moveaxis(out.T.reshape(s.shape), -1, axis)


def interpolate(s, n, bc):
    """Direct transform: c with (Bx (x) By (x) Bz) c = s, one exact 1-D solve per axis."""
    if bc not in (PERIODIC, DIRICHLET):
        raise ValueError("bc must be 'periodic' or 'dirichlet'")
    t = eval_taps(n)
    c = np.asarray(s, dtype=np.float64)
    for axis in (2, 1, 0):
        c = _solve_axis(c, t, axis, bc)
    return c
