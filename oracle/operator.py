"""System operator of the constant-coefficient implicit heat step (oracle; test infrastructure only).

Paper, Sec. 2.4: the tensor form F(c) = t has a diffusion branch c_k d_m w^{klm}, an
absorption branch c_k m_m f^{klm} and a boundary branch; inside the domain the kernels
are shift invariant and separable, w = (1/h^2)(w x f x f + f x w x f + f x f x w) and
f = f x f x f, and the domain computation is the filter cascade of Fig. FiltAlg.

Constant coefficients (D = tau, mu_a = 1 by the partition of unity), no boundary branch,
divided through by h_x h_y h_z (scaling reading, see the design notes):
    A = Mx (x) My (x) Mz + tau * sum_d h_d^-2  (K_d in slot d, M elsewhere)
Arrays are numpy [z, y, x] (x fastest); grid tuples are (Nx, Ny, Nz); h is (hx, hy, hz).

Boundary handling (reading of the homogeneous Dirichlet case): the 1-D Toeplitz bands
are truncated at both ends, i.e. coefficients outside the index box count as zero.
Periodic: circulant bands (requires N_d >= 2n+1, otherwise the taps would alias).
"""
import numpy as np

from .bspline import taps

PERIODIC = "periodic"
DIRICHLET = "dirichlet"

_AXIS = {"x": 2, "y": 1, "z": 0}


def check_args(grid, n, h, tau, bc):
    if bc not in (PERIODIC, DIRICHLET):
        raise ValueError("bc must be 'periodic' or 'dirichlet'")
    if not (1 <= n <= 5):
        raise ValueError("degree n must be in 1..5")
    if tau <= 0 or any(hd <= 0 for hd in h):
        raise ValueError("tau and h must be positive")
    if any(N < 2 * n + 1 for N in grid):
        raise ValueError("every N_d must be >= 2n+1")


def matrix_1d(t, N, bc):
    """Dense N x N banded Toeplitz (Dirichlet: truncated) or circulant (periodic) matrix of taps t."""
    n = (len(t) - 1) // 2
    if bc == PERIODIC and N < 2 * n + 1:
        raise ValueError("periodic band needs N >= 2n+1")
    A = np.zeros((N, N), dtype=np.float64)
    for i in range(N):
        for k in range(-n, n + 1):
            j = i + k
            if bc == PERIODIC:
                A[i, j % N] += t[n + k]
            elif 0 <= j < N:
                A[i, j] += t[n + k]
    return A


def filter_1d(u, t, axis, bc):
    """y_i = sum_k t_k u_{i+k} along one axis of a 3-D array (the 1-D pass of Fig. FiltAlg)."""
    n = (len(t) - 1) // 2
    ax = _AXIS[axis]
    out = np.zeros_like(u, dtype=np.float64)
    N = u.shape[ax]
    for k in range(-n, n + 1):
        if bc == PERIODIC:
            shifted = np.roll(u, -k, axis=ax)
        else:
            shifted = np.zeros_like(u, dtype=np.float64)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if k >= 0:
                src[ax] = slice(k, N)
                dst[ax] = slice(0, N - k)
            else:
                src[ax] = slice(0, N + k)
                dst[ax] = slice(-k, N)
            shifted[tuple(dst)] = u[tuple(src)]
        out += t[n + k] * shifted
    return out


def apply(u, n, h, tau, bc):
    """y = A u, evaluated term by term as in the separable kernel decomposition (12 filter passes)."""
    m, s = taps(n)
    u = np.asarray(u, dtype=np.float64)
    mass = filter_1d(filter_1d(filter_1d(u, m, "x", bc), m, "y", bc), m, "z", bc)
    kx = filter_1d(filter_1d(filter_1d(u, s, "x", bc), m, "y", bc), m, "z", bc)
    ky = filter_1d(filter_1d(filter_1d(u, m, "x", bc), s, "y", bc), m, "z", bc)
    kz = filter_1d(filter_1d(filter_1d(u, m, "x", bc), m, "y", bc), s, "z", bc)
    hx, hy, hz = h
    return mass + tau * (kx / hx ** 2 + ky / hy ** 2 + kz / hz ** 2)


def mass_apply(u, n, bc):
    """(Mx (x) My (x) Mz) u."""
    m, _ = taps(n)
    u = np.asarray(u, dtype=np.float64)
    return filter_1d(filter_1d(filter_1d(u, m, "x", bc), m, "y", bc), m, "z", bc)


def rhs(u_prev, q, n, tau, bc):
    """b = M (u^k + tau q): Galerkin implicit Euler for du/dt = Lap u + f, load vector with n_s = n_b."""
    v = np.asarray(u_prev, dtype=np.float64)
    if q is not None:
        v = v + tau * np.asarray(q, dtype=np.float64)
    return mass_apply(v, n, bc)


def abs_apply(u, n, h, tau, bc):
    """|A| |u| with absolute taps: the scale that bounds the rounding error of any evaluation order of A u."""
    m, s = taps(n)
    m, s = np.abs(m), np.abs(s)
    u = np.abs(np.asarray(u, dtype=np.float64))
    mass = filter_1d(filter_1d(filter_1d(u, m, "x", bc), m, "y", bc), m, "z", bc)
    kx = filter_1d(filter_1d(filter_1d(u, s, "x", bc), m, "y", bc), m, "z", bc)
    ky = filter_1d(filter_1d(filter_1d(u, m, "x", bc), s, "y", bc), m, "z", bc)
    kz = filter_1d(filter_1d(filter_1d(u, m, "x", bc), m, "y", bc), s, "z", bc)
    hx, hy, hz = h
    return mass + tau * (kx / hx ** 2 + ky / hy ** 2 + kz / hz ** 2)


def dense_matrix(grid, n, h, tau, bc):
    """Assembled A as a dense matrix acting on u.ravel() ([z, y, x] C order): only for tiny grids.

    With C-order [z, y, x] flattening, the Kronecker factor order is z (outer), y, x (inner).
    """
    Nx, Ny, Nz = grid
    if Nx * Ny * Nz > 4096:
        raise ValueError("dense assembly is for tiny grids only")
    m, s = taps(n)
    Mx, My, Mz = (matrix_1d(m, N, bc) for N in (Nx, Ny, Nz))
    Kx, Ky, Kz = (matrix_1d(s, N, bc) for N in (Nx, Ny, Nz))
    hx, hy, hz = h
    A = np.kron(Mz, np.kron(My, Mx))
    A = A + tau / hx ** 2 * np.kron(Mz, np.kron(My, Kx))
    A = A + tau / hy ** 2 * np.kron(Mz, np.kron(Ky, Mx))
    A = A + tau / hz ** 2 * np.kron(Kz, np.kron(My, Mx))
    return A
