"""Box domain with the Robin / penalty boundary branch on the GPU against the oracle
(oracle/robin.py): operator and right-hand side elementwise (degrees 1-5, FP64 and FP32, vector
and scalar staging, penalty and moderate gamma), implicit steps against the oracle's fast
diagonalisation, and sampled outputs at 928^3."""
import numpy as np
import pytest

from oracle import bspline, robin
from tests.gpu_util import EPS, dev, host, op_tolerance, rounded
from workloads import normal_field

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")
torch = pytest.importorskip("torch")


def box_h(grid, n):
    """Spacing of the unit box behind N coefficients per axis (Nc = N - 1 - 2 floor(n/2) cells)."""
    return tuple(1.0 / robin.cells(N, n) for N in grid)


def split_abs(N, n, hd, tau, gamma):
    """Per axis, |Toeplitz part| + |corner correction| of the box mass M and of W = tau (h^-2 K +
    h^-1 E / (2 gamma)): the kernels apply the truncated Toeplitz band and add the corner blocks, so
    their rounding is relative to these sums (far above |M| in the nearly empty corner rows of
    degrees 4 and 5)."""
    M, K, E = robin.matrices_1d(N, n)
    W = tau * (K / hd ** 2 + E / (2.0 * gamma * hd))
    m, sk = bspline.taps(n)
    T, S = np.zeros((N, N)), np.zeros((N, N))
    for a in range(-n, n + 1):
        idx = np.arange(max(0, -a), min(N, N - a))
        T[idx, idx + a] = m[n + a]
        S[idx, idx + a] = sk[n + a]
    WT = tau / hd ** 2 * S
    return np.abs(T) + np.abs(M - T), np.abs(WT) + np.abs(W - WT)


def abs_apply(u, n, h, tau, gamma):
    """The rounding scale of A_R u: the abs-split matrices applied to |u|."""
    grid = (u.shape[2], u.shape[1], u.shape[0])
    (Mx, Wx), (My, Wy), (Mz, Wz) = [split_abs(N, n, hd, tau, gamma) for N, hd in zip(grid, h)]
    au = np.abs(u)
    al = lambda A, v, ax: np.moveaxis(np.tensordot(A, v, axes=([1], [ax])), 0, ax)
    return (al(Mz, al(My, al(Mx + Wx, au, 2), 1), 0) + al(Mz, al(Wy, al(Mx, au, 2), 1), 0)
            + al(Wz, al(My, al(Mx, au, 2), 1), 0))


def tol(n, dt, scale):
    """op_tolerance of the filter cascade plus the rounding of the host's FP64 corner tables (each
    an exact quadrature of at most 96 terms): 128 eps relative to the same scale."""
    return op_tolerance(n, dt, scale) + 128 * EPS["f64"] * scale


CASES = [(n, grid, gamma) for n in (1, 2, 3, 4, 5) for grid, gamma in (((20, 18, 17), 1e-3), ((21, 19, 16), 0.7))]


@pytest.mark.parametrize("n,grid,gamma", CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_robin_apply_matches_oracle(n, grid, gamma, dt):
    h, tau = box_h(grid, n), 2e-3
    print("robin apply", n, grid, gamma, dt, flush=True)
    ctx = tbs.RobinContext(grid, n, h, tau, gamma)
    u = rounded(normal_field(grid[::-1], 40 + n), dt)
    y = torch.empty(grid[::-1], dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")
    ctx.apply(dev(u, dt), y)
    ref = robin.apply(u, n, h, tau, gamma)
    bound = tol(n, dt, abs_apply(u, n, h, tau, gamma)) + (np.abs(ref) * 2.0 ** -24 if dt == "f32" else 0.0)
    err = np.abs(host(y) - ref)
    assert np.all(err <= bound), (err.max(), np.unravel_index(np.argmax(err - bound), err.shape))


@pytest.mark.parametrize("n", [1, 3, 4])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_robin_rhs_matches_oracle(n, dt):
    grid, tau = (22, 17, 19), 1e-3
    h = box_h(grid, n)
    ctx = tbs.RobinContext(grid, n, h, tau, 0.05)
    u = rounded(normal_field(grid[::-1], 7), dt)
    q = rounded(normal_field(grid[::-1], 8), dt)
    b = torch.empty(grid[::-1], dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")
    ctx.rhs(dev(u, dt), dev(q, dt), b)
    v = u + (np.float32(tau) * q.astype(np.float32)).astype(np.float64) if dt == "f32" else u + tau * q
    ref = robin.mass_apply(v, n)
    Ma = [split_abs(N, n, 1.0, tau, 0.05)[0] for N in grid]
    al = lambda A, w, ax: np.moveaxis(np.tensordot(A, w, axes=([1], [ax])), 0, ax)
    scale = al(Ma[2], al(Ma[1], al(Ma[0], np.abs(u) + tau * np.abs(q), 2), 1), 0)
    bound = 2 * tol(n, dt, scale) + (np.abs(ref) * 2.0 ** -24 if dt == "f32" else 0.0)
    assert np.all(np.abs(host(b) - ref) <= bound)


def test_robin_operator_is_not_the_truncated_one():
    """The corner blocks change the boundary rows (a kernel that ignored them would pass a test
    whose field vanishes near the faces)."""
    grid, n, tau, gamma = (20, 18, 17), 3, 2e-3, 1e-3
    h = box_h(grid, n)
    u = normal_field(grid[::-1], 3)
    yr = torch.empty(grid[::-1], dtype=torch.float64, device="cuda")
    yd = torch.empty_like(yr)
    tbs.RobinContext(grid, n, h, tau, gamma).apply(dev(u), yr)
    tbs.Context(grid, n, h, tau, "dirichlet").apply(dev(u), yd)
    d = np.abs(host(yr) - host(yd))
    assert d[:, :, 0].max() > 1e-2 and d[3:-3, 3:-3, 3:-3].max() < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("gamma", [1e-3, 0.5])
def test_robin_timestep_matches_fast_diagonalisation(prec, gamma):
    # linear B-splines (the leg example's degree): A_R is well conditioned (kappa ~ 20-30); from
    # degree 2 on the box's nearly empty corner B-splines make it ill conditioned (kappa ~ 1e8 at
    # 12^3), which unpreconditioned CG resolves only slowly
    grid, n, tau = (16, 16, 15), 1, 1e-3  # small enough for the dense condition number
    h = box_h(grid, n)
    ctx = tbs.RobinContext(grid, n, h, tau, gamma)
    p = {"fp64": tbs.PREC_FP64, "mixed": tbs.PREC_MIXED}[prec]
    ctx.ensure_workspace(p)
    u0, q = normal_field(grid[::-1], 21), normal_field(grid[::-1], 22)
    un = torch.empty(grid[::-1], dtype=torch.float64, device="cuda")
    rtol = 1e-11
    st = ctx.timestep(dev(u0), dev(q), un, p, rtol, 2000)
    assert st["converged"], st
    got = host(un)
    b = robin.rhs(u0, q, n, tau)
    res = np.linalg.norm(b - robin.apply(got, n, h, tau, gamma)) / np.linalg.norm(b)
    assert res <= 2 * rtol, res
    ref = robin.step(u0, q, n, h, tau, gamma)
    ev = np.linalg.eigvalsh(robin.dense_matrix(grid, n, h, tau, gamma))
    kappa = ev[-1] / ev[0]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 2 * kappa * rtol, (err, kappa)


@pytest.mark.parametrize("n", [2, 3])
def test_robin_cg_reduces_the_residual_at_higher_degree(n):
    # cubic / quadratic box: FP64 CG through the C ABI on the Robin operator; the recursive residual
    # it reports agrees with the oracle's residual of its iterate
    grid, tau, gamma = (20, 18, 17), 1e-3, 0.05
    h = box_h(grid, n)
    ctx = tbs.RobinContext(grid, n, h, tau, gamma)
    ctx.ensure_workspace(tbs.PREC_FP64)
    u0 = normal_field(grid[::-1], 23)
    b = robin.rhs(u0, None, n, tau)
    x = dev(u0)
    ctx.cg_begin(dev(b), x, 1e-6)
    rel, it = ctx.cg_step(300)
    got = host(x)
    true_rel = np.linalg.norm(b - robin.apply(got, n, h, tau, gamma)) / np.linalg.norm(b)
    rel0 = np.linalg.norm(b - robin.apply(u0, n, h, tau, gamma)) / np.linalg.norm(b)
    assert true_rel < 0.01 * rel0
    assert abs(true_rel - rel) <= 1e-3 * rel0


@pytest.mark.parametrize("n", [4, 5])
@pytest.mark.parametrize("fused", [1, 0])
def test_robin_fp64_cg_iterates_at_degrees_4_and_5(n, fused):
    # quartic / quintic box: the one-kernel FP64 iteration falls back to 8-row tiles there (the
    # 16-row one would not fit its LDS); its first iterates and residual history against the
    # oracle's Hestenes-Stiefel CG on the Robin operator, and against the two-kernel form
    from oracle import solvers
    grid, tau, gamma, k = (21, 19, 18), 1e-3, 0.05, 4
    h = box_h(grid, n)
    ctx = tbs.RobinContext(grid, n, h, tau, gamma)
    ctx.set_opts(fused_cg=fused)
    ctx.ensure_workspace(tbs.PREC_FP64)
    x0 = normal_field(grid[::-1], 31) * 0.1
    b = normal_field(grid[::-1], 32)
    x = dev(x0)
    ctx.cg_begin(dev(b), x, 0.0)
    rel, it = ctx.cg_step(k)
    xr, _, hist = solvers.cg(lambda v: robin.apply(v, n, h, tau, gamma), b, x0, 0.0, 100, fixed_iters=k)
    assert it == k
    assert np.linalg.norm(host(x) - xr) <= 1e-9 * np.linalg.norm(xr)
    assert abs(rel - hist[-1]) <= 1e-7 * hist[-1]


def test_robin_apply_928_sampled():
    n, N, tau, gamma = 3, 928, 1e-5, 1e-3
    grid = (N, N, N)
    h = box_h(grid, n)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    u = torch.randn((N, N, N), generator=g, device="cuda", dtype=torch.float64)
    ctx = tbs.RobinContext(grid, n, h, tau, gamma)
    M, K, E = robin.matrices_1d(N, n)  # every axis has the same size and spacing
    W = tau * (K / h[0] ** 2 + E / (2.0 * gamma * h[0]))
    Ma, Wa = split_abs(N, n, h[0], tau, gamma)
    for dt in ("f64", "f32"):
        src = u if dt == "f64" else u.float()
        y = torch.empty((N, N, N), dtype=src.dtype, device="cuda")
        ctx.apply(src, y)
        rng = np.random.default_rng(9)
        pts = [tuple(rng.integers(0, N, 3)) for _ in range(400)]
        for a in (0, 1, 2, 3, 4, 63, 64, N // 2, N - 5, N - 4, N - 3, N - 2, N - 1):
            pts += [(a, a, a), (0, a, N - 1), (a, 2, 5), (N - 1, a, 1)]
        pts = np.array(pts)
        got = y[tuple(torch.from_numpy(pts.T).cuda())].to(torch.float64).cpu().numpy()
        for (k, j, i), gv in zip(pts, got):
            sl = [slice(max(c - n, 0), min(c + n + 1, N)) for c in (k, j, i)]
            blk = src[sl[0], sl[1], sl[2]].to(torch.float64).cpu().numpy()
            mz, my, mx = (M[c, s] for c, s in zip((k, j, i), sl))
            wz, wy, wx = (W[c, s] for c, s in zip((k, j, i), sl))
            ref = (np.einsum("c,b,a,cba->", mz, my, mx + wx, blk) + np.einsum("c,b,a,cba->", mz, wy, mx, blk)
                   + np.einsum("c,b,a,cba->", wz, my, mx, blk))
            az, ay, ax_ = (Ma[c, s_] for c, s_ in zip((k, j, i), sl))
            bz, by, bx = (Wa[c, s_] for c, s_ in zip((k, j, i), sl))
            ab = np.abs(blk)
            sc = (np.einsum("c,b,a,cba->", az, ay, ax_ + bx, ab) + np.einsum("c,b,a,cba->", az, by, ax_, ab)
                  + np.einsum("c,b,a,cba->", bz, ay, ax_, ab))
            bound = tol(n, dt, sc) + (abs(ref) * 2.0 ** -24 if dt == "f32" else 0.0)
            assert abs(gv - ref) <= bound, ((k, j, i), dt, gv, ref)
        del y
