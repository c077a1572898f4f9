"""Exact (direct) solutions of one implicit step A u^{k+1} = b (oracle; test infrastructure only).

These do not use CG, so they pin the iterative path from outside.

Periodic: A is a sum of Kronecker products of circulants, hence diagonal in the 3-D DFT
basis; with the 1-D symbols M(w), K(w) of the mass and stiffness taps the step is
    u^{k+1}^(w) = (u^k + tau q)^(w) * g(w),  g = 1 / (1 + tau * sum_d K(w_d) / (h_d^2 M(w_d))).
Dirichlet (truncated bands): fast diagonalisation (Lynch, Rice & Thomas 1964): per axis solve
the generalised symmetric eigenproblem K_d V_d = M_d V_d L_d with V_d^T M_d V_d = I, then
V^T A V = I + tau * sum_d L_d / h_d^2 with V = Vx (x) Vy (x) Vz.
"""
import numpy as np
import scipy.linalg

from .bspline import symbol_from_taps, taps
from .operator import DIRICHLET, PERIODIC, matrix_1d, rhs


def decay_factors(grid, n, h, tau):
    """g(w) on the DFT grid, array [z, y, x] (periodic case)."""
    m, s = taps(n)
    Nx, Ny, Nz = grid
    hx, hy, hz = h
    terms = 0.0
    for N, hd, ax in ((Nx, hx, 2), (Ny, hy, 1), (Nz, hz, 0)):
        w = 2.0 * np.pi * np.arange(N) / N
        ratio = symbol_from_taps(s, w) / (hd * hd * symbol_from_taps(m, w))
        shape = [1, 1, 1]
        shape[ax] = N
        terms = terms + ratio.reshape(shape)
    return 1.0 / (1.0 + tau * terms)


def solve_periodic(b, n, h, tau):
    """u = A^-1 b for periodic BC by the 3-D FFT (b is any right-hand side)."""
    m, s = taps(n)
    Nz, Ny, Nx = b.shape
    hx, hy, hz = h
    sym = 1.0
    for N, hd, ax in ((Nx, hx, 2), (Ny, hy, 1), (Nz, hz, 0)):
        w = 2.0 * np.pi * np.arange(N) / N
        shape = [1, 1, 1]
        shape[ax] = N
        mw = symbol_from_taps(m, w).reshape(shape)
        kw = symbol_from_taps(s, w).reshape(shape)
        sym = sym * mw  # mass symbol product
    a_sym = sym.copy()
    for N, hd, ax in ((Nx, hx, 2), (Ny, hy, 1), (Nz, hz, 0)):
        w = 2.0 * np.pi * np.arange(N) / N
        shape = [1, 1, 1]
        shape[ax] = N
        a_sym = a_sym + tau / hd ** 2 * sym * (symbol_from_taps(s, w) / symbol_from_taps(m, w)).reshape(shape)
    return np.real(np.fft.ifftn(np.fft.fftn(b) / a_sym))


def step_periodic(u_prev, q, n, h, tau):
    """Exact implicit Euler step, periodic, via the per-mode decay factor g(w)."""
    v = np.asarray(u_prev, dtype=np.float64)
    if q is not None:
        v = v + tau * q
    Nz, Ny, Nx = v.shape
    g = decay_factors((Nx, Ny, Nz), n, h, tau)
    return np.real(np.fft.ifftn(np.fft.fftn(v) * g))


def _gen_eig(n, N):
    m, s = taps(n)
    M = matrix_1d(m, N, DIRICHLET)
    K = matrix_1d(s, N, DIRICHLET)
    lam, V = scipy.linalg.eigh(K, M)
    return lam, V


def solve_dirichlet(b, n, h, tau):
    """u = A^-1 b for truncated (Dirichlet) bands by fast diagonalisation."""
    Nz, Ny, Nx = b.shape
    hx, hy, hz = h
    lx, Vx = _gen_eig(n, Nx)
    ly, Vy = _gen_eig(n, Ny)
    lz, Vz = _gen_eig(n, Nz)
    # c = V^T b: contract each axis with V_d^T
    c = np.einsum("ia,zyi->zya", Vx, b)
    c = np.einsum("ja,zjx->zax", Vy, c)
    c = np.einsum("ka,kyx->ayx", Vz, c)
    d = 1.0 + tau * (lz[:, None, None] / hz ** 2 + ly[None, :, None] / hy ** 2 + lx[None, None, :] / hx ** 2)
    c = c / d
    u = np.einsum("ia,zya->zyi", Vx, c)
    u = np.einsum("ja,zax->zjx", Vy, u)
    u = np.einsum("ka,ayx->kyx", Vz, u)
    return u


def step(u_prev, q, n, h, tau, bc):
    """Exact implicit Euler step u^{k+1} = A^-1 M (u^k + tau q) for either boundary condition."""
    if bc == PERIODIC:
        return step_periodic(u_prev, q, n, h, tau)
    b = rhs(u_prev, q, n, tau, bc)
    return solve_dirichlet(b, n, h, tau)


def solve(b, n, h, tau, bc):
    if bc == PERIODIC:
        return solve_periodic(b, n, h, tau)
    return solve_dirichlet(b, n, h, tau)


def condition_number(grid, n, h, tau, bc, samples=129):
    """kappa(A).  Periodic: exact, from the symbol on the DFT grid.  Dirichlet (truncated bands):
    A is a symmetric three-level Toeplitz matrix, and x^T A x is the integral of its generating
    symbol a(w) against |x^(w)|^2, so every eigenvalue lies in [min a, max a]; the ratio of the
    symbol's extremes (sampled finely on [0, pi]^3, where a is even in each w_d) bounds kappa."""
    m, s = taps(n)
    if bc == PERIODIC:
        ws = [2.0 * np.pi * np.arange(N) / N for N in grid]
    else:
        ws = [np.linspace(0.0, np.pi, samples) for _ in grid]
    lam = 1.0
    tot = 1.0
    for w, hd, ax in zip(ws, h, (2, 1, 0)):
        shape = [1, 1, 1]
        shape[ax] = len(w)
        mw = symbol_from_taps(m, w)
        lam = lam * mw.reshape(shape)
        tot = tot + tau / hd ** 2 * (symbol_from_taps(s, w) / mw).reshape(shape)
    a = lam * tot
    return float(a.max() / a.min())
