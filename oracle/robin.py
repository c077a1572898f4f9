"""Box-domain Robin / penalty boundary branch of the system operator (oracle; test infrastructure only).

Paper, Sec. 2.2: for the Robin condition  2 D dphi/dn + phi = 0  integration by parts adds the
boundary branch (1/2) int_{dOmega} phi psi ds to the bilinear form a(.,.); Sec. 2.3, discrete
Ritz-Galerkin system: that branch enters as (1/(2 gamma)) sum_k c_k int_{dOmega} b_k b_l ds, and
every domain integral is taken over Omega only; Sec. 2.4: the boundary tensor h^{kl} of the tensor
form F(c) = t.  With a small gamma the branch imposes phi = 0 weakly (the Dirichlet-by-penalty of
the Sec. 3 leg example).

Domain and basis (box reading): Omega = [0, Lx] x [0, Ly] x [0, Lz], L_d = Nc_d h_d (Nc_d whole
cells), and every B-spline b^n(x/h - k) whose support meets the open box is a basis function,
i.e. k = -floor(n/2) .. Nc + floor(n/2): N_d = Nc_d + 1 + 2 floor(n/2) coefficients per axis (the
basis count behind Table tblFlop1d).  Array index i holds offset k = i - floor(n/2).  On a box the
integrals factor per axis (Table 1 scalar-product row restricted to [0, Nc], derivative row):
    M~[i,j] = int_0^Nc b(x-k_i) b(x-k_j) dx,   K~[i,j] = int_0^Nc b'(x-k_i) b'(x-k_j) dx,
    E[i,j]  = b(-k_i) b(-k_j) + b(Nc-k_i) b(Nc-k_j)       (the two end points of the axis),
and, divided through by hx hy hz like the rest of the operator (a face x = 0 contributes
h_y h_z E_x M~_y M~_z before the division), one implicit Euler step of du/dt = Lap u + f with
du/dn + u / (2 gamma) = 0 on the boundary solves
    A_R u^{k+1} = M~x M~y M~z (u^k + tau q),
    A_R = M~x M~y M~z + tau * sum_d (h_d^-2 K~_d + h_d^-1 E_d / (2 gamma))  [slot d; M~ elsewhere].
Inside the box the rows are the Toeplitz rows of the constant-coefficient operator; only rows
within 2 floor(n/2) of an end differ.  The integrals are computed exactly (up to rounding) by
Gauss-Legendre quadrature with n+1 points on every polynomial piece (products of two degree-n
pieces have degree 2n <= 2(n+1) - 1).
"""
import numpy as np
import scipy.linalg

from numpy.polynomial.legendre import leggauss


def bspline_f(p, x):
    """Centred B-spline b^p at float points x (numpy), by the truncated-power expansion of the
    (p+1)-fold box convolution (Table 1 convolution row); p = 0 is the box on (-1/2, 1/2]."""
    from math import comb, factorial
    x = np.asarray(x, dtype=np.float64)
    half = 0.5 * (p + 1)
    # b^p is even: evaluating at -|x| keeps only the few truncated powers that are positive near
    # the left end of the support, which avoids cancellation in the tails
    xn = -np.abs(x)
    acc = np.zeros_like(x)
    for j in range(p + 2):
        t = xn + half - j
        if p == 0:
            tp = (t > 0).astype(np.float64)
        else:
            tp = np.where(t > 0, t, 0.0) ** p
        acc = acc + (-1) ** j * comb(p + 1, j) * tp
    out = acc / factorial(p)
    return np.where(np.abs(x) < half, out, 0.0)


def bspline_d(p, x):
    """b^p'(x) = b^{p-1}(x + 1/2) - b^{p-1}(x - 1/2)  (Table 1 derivative row), p >= 1."""
    x = np.asarray(x, dtype=np.float64)
    return bspline_f(p - 1, x + 0.5) - bspline_f(p - 1, x - 0.5)


def cells(N, n):
    """Whole cells Nc of the box behind N coefficients of degree n."""
    nc = N - 1 - 2 * (n // 2)
    if nc < 1:
        raise ValueError("too few coefficients for degree %d" % n)
    return nc


def offsets(N, n):
    """B-spline offsets k of the N basis functions (array index i <-> k = i - floor(n/2))."""
    return np.arange(N) - n // 2


def _breakpoints(nc, n):
    # knots of b^n(x - k): integers for odd n, half-integers for even n; plus the box ends
    if n % 2:
        return np.arange(0, nc + 1, dtype=np.float64)
    return np.concatenate([[0.0], np.arange(0.5, nc, 1.0), [float(nc)]])


def matrices_1d(N, n):
    """(M~, K~, E) for N coefficients of degree n on the box [0, Nc] (unit spacing)."""
    nc = cells(N, n)
    k = offsets(N, n).astype(np.float64)
    xg, wg = leggauss(n + 1)
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    br = _breakpoints(nc, n)
    for a, b in zip(br[:-1], br[1:]):
        x = 0.5 * (a + b) + 0.5 * (b - a) * xg
        w = 0.5 * (b - a) * wg
        B = bspline_f(n, x[None, :] - k[:, None])
        D = bspline_d(n, x[None, :] - k[:, None])
        M += (B * w) @ B.T
        K += (D * w) @ D.T
    b0 = bspline_f(n, 0.0 - k)
    b1 = bspline_f(n, nc - k)
    E = np.outer(b0, b0) + np.outer(b1, b1)
    return M, K, E


def axis_matrices(grid, n, h, tau, gamma):
    """Per axis (x, y, z): (M~_d, W_d) with W_d = tau (h_d^-2 K~_d + h_d^-1 E_d / (2 gamma))."""
    out = []
    for N, hd in zip(grid, h):
        M, K, E = matrices_1d(N, n)
        out.append((M, tau * (K / hd ** 2 + E / (2.0 * gamma * hd))))
    return out


def _along(Amat, u, axis):
    # y[..., i, ...] = sum_j Amat[i, j] u[..., j, ...] along array axis `axis` of [z, y, x]
    return np.moveaxis(np.tensordot(Amat, u, axes=([1], [axis])), 0, axis)


def apply(u, n, h, tau, gamma):
    """y = A_R u (u is [z, y, x]); each Kronecker term applied by 1-D matrix products."""
    u = np.asarray(u, dtype=np.float64)
    grid = (u.shape[2], u.shape[1], u.shape[0])
    (Mx, Wx), (My, Wy), (Mz, Wz) = axis_matrices(grid, n, h, tau, gamma)
    ax = {"x": 2, "y": 1, "z": 0}
    mass = _along(Mz, _along(My, _along(Mx, u, ax["x"]), ax["y"]), ax["z"])
    tx = _along(Mz, _along(My, _along(Wx, u, ax["x"]), ax["y"]), ax["z"])
    ty = _along(Mz, _along(Wy, _along(Mx, u, ax["x"]), ax["y"]), ax["z"])
    tz = _along(Wz, _along(My, _along(Mx, u, ax["x"]), ax["y"]), ax["z"])
    return mass + tx + ty + tz


def mass_apply(u, n):
    """M~x M~y M~z u."""
    u = np.asarray(u, dtype=np.float64)
    out = u
    for N, axis in ((u.shape[2], 2), (u.shape[1], 1), (u.shape[0], 0)):
        M, _, _ = matrices_1d(N, n)
        out = _along(M, out, axis)
    return out


def rhs(u_prev, q, n, tau):
    v = np.asarray(u_prev, dtype=np.float64)
    if q is not None:
        v = v + tau * np.asarray(q, dtype=np.float64)
    return mass_apply(v, n)


def dense_matrix(grid, n, h, tau, gamma):
    """Assembled A_R acting on u.ravel() ([z, y, x] C order): tiny grids only."""
    Nx, Ny, Nz = grid
    if Nx * Ny * Nz > 4096:
        raise ValueError("dense assembly is for tiny grids only")
    (Mx, Wx), (My, Wy), (Mz, Wz) = axis_matrices(grid, n, h, tau, gamma)
    k = np.kron
    return k(Mz, k(My, Mx)) + k(Mz, k(My, Wx)) + k(Mz, k(Wy, Mx)) + k(Wz, k(My, Mx))


def solve(b, n, h, tau, gamma):
    """u = A_R^-1 b by fast diagonalisation: per axis W_d V_d = M~_d V_d L_d, V_d^T M~_d V_d = I."""
    Nz, Ny, Nx = b.shape
    eig = []
    for M, W in axis_matrices((Nx, Ny, Nz), n, h, tau, gamma):
        eig.append(scipy.linalg.eigh(W, M))
    (lx, Vx), (ly, Vy), (lz, Vz) = eig
    c = np.einsum("ia,zyi->zya", Vx, b)
    c = np.einsum("ja,zjx->zax", Vy, c)
    c = np.einsum("ka,kyx->ayx", Vz, c)
    c = c / (1.0 + lz[:, None, None] + ly[None, :, None] + lx[None, None, :])
    u = np.einsum("ia,zya->zyi", Vx, c)
    u = np.einsum("ja,zax->zjx", Vy, u)
    return np.einsum("ka,ayx->kyx", Vz, u)


def step(u_prev, q, n, h, tau, gamma):
    return solve(rhs(u_prev, q, n, tau), n, h, tau, gamma)
