"""Variable-coefficient system operator (oracle; test infrastructure only).

Paper, Sec. 2.3: the diffusion coefficient D(x) and the absorption coefficient mu_a(x) are expanded
in the same B-spline basis as the solution, D = sum_m d_m b_m, mu_a = sum_m m_m b_m (n_p = n_b = n),
and the discrete Ritz-Galerkin system has the domain branches
    sum_k c_k sum_m d_m int grad b_k . grad b_l b_m dx  +  sum_k c_k sum_m m_m int b_k b_l b_m dx;
Sec. 2.4: in tensor form c_k d_m w^{klm} + c_k m_m f^{klm}, with the shift-invariant separable
three-index kernels  f = f^ x f^ x f^  and  w = h_x^-2 w^ x f^ x f^ + h_y^-2 f^ x w^ x f^ + h_z^-2 f^ x f^ x w^
(the 1/h^2 factors of the separable kernel decomposition), where, in units of the grid spacing,
    f^(k, l, m) = int b(x-k) b(x-l) b(x-m) dx,   w^(k, l, m) = int b'(x-k) b'(x-l) b(x-m) dx,
which depend on k - m and l - m only.  Divided through by hx hy hz like the constant-coefficient
operator, F(c)_l = sum_k sum_m c_k (m_m f^{klm} + d_m w^{klm}).

With d = tau and m = 1 everywhere, sum_m f^(k, l, m) = m_{k-l} and sum_m w^(k, l, m) = s_{k-l}
(partition of unity), so F = A, the implicit-step operator.

Boundary readings: periodic grids wrap every index; on a truncated (Dirichlet) grid the unknown
c is zero outside the index box, as for A, and the coefficient fields d, m continue beyond it by
their edge values (D and mu_a stay the B-spline expansions of the box's edge coefficients, so
constant coefficients give exactly A there too).

The 1-D kernels are integrated exactly (up to rounding) by Gauss-Legendre quadrature on every
polynomial piece: the product of three degree-n pieces has degree 3n, and ceil((3n+1)/2) points
integrate it exactly.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss

from .robin import bspline_d, bspline_f

_AX = {"x": 2, "y": 1, "z": 0}


def kernels_1d(n):
    """(F, W): arrays [p + n, q + n] for p = k - m, q = l - m in -n..n:
    F[p, q] = int b(x-p) b(x-q) b(x) dx,  W[p, q] = int b'(x-p) b'(x-q) b(x) dx  (unit spacing)."""
    hs = 0.5 * (n + 1)
    npts = (3 * n + 2) // 2
    xg, wg = leggauss(npts)
    br = np.arange(-hs, hs + 0.5, 1.0)  # knots of b(x): integers (odd n) or half-integers (even n)
    F = np.zeros((2 * n + 1, 2 * n + 1))
    W = np.zeros((2 * n + 1, 2 * n + 1))
    for p in range(-n, n + 1):
        for q in range(-n, n + 1):
            acc_f = acc_w = 0.0
            for a, b in zip(br[:-1], br[1:]):
                x = 0.5 * (a + b) + 0.5 * (b - a) * xg
                w = 0.5 * (b - a) * wg
                bm = bspline_f(n, x)
                acc_f += np.sum(w * bspline_f(n, x - p) * bspline_f(n, x - q) * bm)
                acc_w += np.sum(w * bspline_d(n, x - p) * bspline_d(n, x - q) * bm)
            F[p + n, q + n] = acc_f
            W[p + n, q + n] = acc_w
    return F, W


def _shift(v, s, axis, bc, fill):
    """out[i] = v[i + s] along `axis`: wrapped (periodic) or, beyond the box, `fill` ("zero" or
    "edge": the nearest in-box value)."""
    if bc == "periodic":
        return np.roll(v, -s, axis=axis)
    N = v.shape[axis]
    idx = np.arange(N) + s
    inside = (idx >= 0) & (idx < N)
    out = np.take(v, np.clip(idx, 0, N - 1), axis=axis)
    if fill == "zero":
        shape = [1, 1, 1]
        shape[axis] = N
        out = out * inside.reshape(shape)
    return out


def _filter(v, taps, axis, bc):
    """sum over a of taps[a + n] * v[i + a] along axis (c zero outside a truncated box)."""
    n = (len(taps) - 1) // 2
    out = np.zeros_like(v)
    for a in range(-n, n + 1):
        if taps[a + n] != 0.0:
            out += taps[a + n] * _shift(v, a, axis, bc, "zero")
    return out


def apply(c, d, m, n, h, bc):
    """F(c)_l = sum_k sum_m c_k (m_m f^{klm} + d_m w^{klm}) for [z, y, x] arrays c, d, m.

    With beta = m - l and alpha = k - l the kernel factor of axis j is K_j(alpha_j - beta_j, -beta_j);
    for every beta the sum over alpha is a separable filter of c (the shift-invariant separable
    kernels of Sec. 2.4 applied per coefficient index):
        F(c)_l = sum_beta [ m_{l+beta} G_beta(l) + d_{l+beta} H_beta(l) ],
        G_beta = (f_bx (x) f_by (x) f_bz) c,
        H_beta = (hx^-2 w_bx f_by f_bz + hy^-2 f_bx w_by f_bz + hz^-2 f_bx f_by w_bz) c,
    with the 1-D taps f_b(alpha) = F^(alpha - b, -b), w_b(alpha) = W^(alpha - b, -b)."""
    c = np.asarray(c, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    F, W = kernels_1d(n)
    hx, hy, hz = h

    def taps(K, b):
        t = np.zeros(2 * n + 1)
        for a in range(-n, n + 1):
            if abs(a - b) <= n:
                t[a + n] = K[a - b + n, -b + n]
        return t

    out = np.zeros_like(c)
    for bz in range(-n, n + 1):
        cz_f = _filter(c, taps(F, bz), _AX["z"], bc)
        cz_w = _filter(c, taps(W, bz), _AX["z"], bc)
        for by in range(-n, n + 1):
            fy, wy = taps(F, by), taps(W, by)
            ff = _filter(cz_f, fy, _AX["y"], bc)   # f_by f_bz
            fw = _filter(cz_w, fy, _AX["y"], bc)   # f_by w_bz
            wf = _filter(cz_f, wy, _AX["y"], bc)   # w_by f_bz
            for bx in range(-n, n + 1):
                fx, wx = taps(F, bx), taps(W, bx)
                G = _filter(ff, fx, _AX["x"], bc)
                H = (_filter(ff, wx, _AX["x"], bc) / hx ** 2 + _filter(wf, fx, _AX["x"], bc) / hy ** 2
                     + _filter(fw, fx, _AX["x"], bc) / hz ** 2)
                ms = _shift(_shift(_shift(m, bx, _AX["x"], bc, "edge"), by, _AX["y"], bc, "edge"), bz, _AX["z"], bc, "edge")
                ds = _shift(_shift(_shift(d, bx, _AX["x"], bc, "edge"), by, _AX["y"], bc, "edge"), bz, _AX["z"], bc, "edge")
                out += ms * G + ds * H
    return out


def dense_matrix(grid, d, m, n, h, bc):
    """A[l, k] = sum_m (m_m f^{klm} + d_m w^{klm}) assembled entry by entry from the three-index
    kernels (explicit loops; tiny grids only).  Coefficient indices beyond a truncated box take the
    edge value; periodic indices wrap."""
    Nx, Ny, Nz = grid
    if Nx * Ny * Nz > 512:
        raise ValueError("dense assembly is for tiny grids only")
    F, W = kernels_1d(n)
    hx, hy, hz = h
    d = np.asarray(d, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    N = Nx * Ny * Nz
    A = np.zeros((N, N))

    def coef(arr, i, j, k):
        if bc == "periodic":
            return arr[k % Nz, j % Ny, i % Nx]
        return arr[min(max(k, 0), Nz - 1), min(max(j, 0), Ny - 1), min(max(i, 0), Nx - 1)]

    def wrap(i, Nd):
        if bc == "periodic":
            return i % Nd
        return i if 0 <= i < Nd else None

    def k1(K, p, q):
        return K[p + n, q + n] if abs(p) <= n and abs(q) <= n else 0.0

    for lz in range(Nz):
        for ly in range(Ny):
            for lx in range(Nx):
                row = (lz * Ny + ly) * Nx + lx
                for ax in range(-n, n + 1):
                    kx = wrap(lx + ax, Nx)
                    for ay in range(-n, n + 1):
                        ky = wrap(ly + ay, Ny)
                        for az in range(-n, n + 1):
                            kz = wrap(lz + az, Nz)
                            if kx is None or ky is None or kz is None:
                                continue
                            col = (kz * Ny + ky) * Nx + kx
                            acc = 0.0
                            for bx in range(-n, n + 1):
                                for by in range(-n, n + 1):
                                    for bz in range(-n, n + 1):
                                        fx, fy, fz = k1(F, ax - bx, -bx), k1(F, ay - by, -by), k1(F, az - bz, -bz)
                                        wx, wy, wz = k1(W, ax - bx, -bx), k1(W, ay - by, -by), k1(W, az - bz, -bz)
                                        mm = coef(m, lx + bx, ly + by, lz + bz)
                                        dd = coef(d, lx + bx, ly + by, lz + bz)
                                        acc += mm * fx * fy * fz + dd * (wx * fy * fz / hx ** 2 + fx * wy * fz / hy ** 2
                                                                         + fx * fy * wz / hz ** 2)
                            A[row, col] += acc
    return A
