"""Coarse-grid initial guess (oracle; test infrastructure only).

Sec. 3, leg example: CG starts from a solution computed on a reduced grid.  Reading: the reduced
grid halves every axis.  For odd degree n the coarse B-spline space lies inside the fine one by the
two-scale relation beta^n(x/2) = 2^-n sum_k C(n+1, k + (n+1)/2) beta^n(x - k), k = -(n+1)/2 ..
(n+1)/2 (a consequence of the convolution row of Table 1: beta^n is n+1 box functions convolved,
and a box of width 2 is two boxes of width 1), so a coarse spline is carried to the fine grid by
the prolongation P, c_i = sum_j C_j w_{i - p(j)}, with p(j) the fine index of coarse node j.  The
coarse system is the Galerkin projection P^T A P / 8 (the operator is normalised by 1/(hx hy hz)),
which is the same operator rediscretised with spacing 2h where the spaces nest (everywhere on an
even periodic grid, away from the ends of a Dirichlet one).  The guess is x0 = u + P d with
A_c d = P^T (b - A u) / 8 solved by CG to a loose tolerance.

Geometry: Dirichlet, p(j) = 2j + 1 and Nc = N // 2 (the truncated band drops the coefficients
that would fall outside the box); periodic, N even, p(j) = 2j and Nc = N / 2.  Arrays numpy
[z, y, x], grids (Nx, Ny, Nz).
"""
from math import comb

import numpy as np

from . import operator as op
from . import solvers


def weights(n):
    """Two-scale weights w_k, k = -(n+1)/2 .. (n+1)/2, for odd degree n."""
    if n % 2 == 0 or not (1 <= n <= 5):
        raise ValueError("the dyadic coarse space nests for odd degrees 1, 3, 5 only")
    H = (n + 1) // 2
    return {k: comb(n + 1, k + H) / 2.0 ** n for k in range(-H, H + 1)}


def coarse_grid(grid, bc):
    if bc == op.PERIODIC:
        if any(N % 2 for N in grid):
            raise ValueError("a periodic coarse grid needs even sizes")
        return tuple(N // 2 for N in grid)
    return tuple(N // 2 for N in grid)


def _offset(bc):
    return 0 if bc == op.PERIODIC else 1


def prolong_1d(C, N, axis, n, bc):
    """Coarse -> fine along one axis: c_i = sum_j C_j w_{i - p(j)}."""
    w = weights(n)
    off = _offset(bc)
    C = np.moveaxis(np.asarray(C, dtype=np.float64), axis, -1)
    out = np.zeros(C.shape[:-1] + (N,))
    for j in range(C.shape[-1]):
        for k, wk in w.items():
            i = 2 * j + off + k
            if bc == op.PERIODIC:
                out[..., i % N] += wk * C[..., j]
            elif 0 <= i < N:
                out[..., i] += wk * C[..., j]
    return np.moveaxis(out, -1, axis)


def restrict_1d(f, Nc, axis, n, bc):
    """Fine -> coarse along one axis, the adjoint of prolong_1d: F_j = sum_k w_k f_{p(j) + k}."""
    w = weights(n)
    off = _offset(bc)
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, -1)
    N = f.shape[-1]
    out = np.zeros(f.shape[:-1] + (Nc,))
    for j in range(Nc):
        for k, wk in w.items():
            i = 2 * j + off + k
            if bc == op.PERIODIC:
                out[..., j] += wk * f[..., i % N]
            elif 0 <= i < N:
                out[..., j] += wk * f[..., i]
    return np.moveaxis(out, -1, axis)


def prolong(C, grid, n, bc):
    for axis, N in ((2, grid[0]), (1, grid[1]), (0, grid[2])):
        C = prolong_1d(C, N, axis, n, bc)
    return C


def restrict(f, grid, n, bc):
    gc = coarse_grid(grid, bc)
    for axis, Nc in ((2, gc[0]), (1, gc[1]), (0, gc[2])):
        f = restrict_1d(f, Nc, axis, n, bc)
    return f


def guess(u, b, n, h, tau, bc, coarse_rtol, max_iter=500):
    """x0 = u + P d, A_c d = P^T (b - A u) / 8 by CG from d = 0 to coarse_rtol; returns (x0, iterations)."""
    grid = u.shape[::-1]
    gc = coarse_grid(grid, bc)
    hc = tuple(2.0 * hd for hd in h)
    r0 = b - op.apply(u, n, h, tau, bc)
    bc_ = restrict(r0, grid, n, bc) / 8.0
    d, it, _ = solvers.cg(lambda v: op.apply(v, n, hc, tau, bc), bc_, np.zeros(gc[::-1]), coarse_rtol, max_iter)
    return u + prolong(d, grid, n, bc), it
