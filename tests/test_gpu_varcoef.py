"""Variable-coefficient operator on the GPU (tbs_apply_varcoef) against the oracle
(oracle/varcoef.py: three-index kernels by exact quadrature, applied as per-offset separable
filters): elementwise at small sizes for degrees 1-5, both boundary conditions, FP64 and FP32;
reduction to the constant-coefficient operator; run-to-run bitwise reproducibility; and sampled
outputs at 928^3."""
import numpy as np
import pytest

from oracle import operator as op, varcoef
from tests.gpu_util import EPS, dev, host, rounded
from workloads import normal_field

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")
torch = pytest.importorskip("torch")


def coef_fields(shape, seed, tau):
    """A positive diffusion field of size tau and a positive absorption field of size 1."""
    d = tau * (1.0 + 0.5 * np.tanh(normal_field(shape, seed)))
    m = 1.0 + 0.5 * np.tanh(normal_field(shape, seed + 1))
    return d, m


def abs_scale(c, d, m, n, h, bc, monkeypatch):
    """sum_k sum_m |c_k| (|m_m| |f^klm| + |d_m| |w^klm|): the oracle's apply on absolute values
    with absolute kernels (the scale of a rounding bound)."""
    F, W = varcoef.kernels_1d(n)
    with monkeypatch.context() as mp:
        mp.setattr(varcoef, "kernels_1d", lambda n_: (np.abs(F), np.abs(W)))
        return varcoef.apply(np.abs(c), np.abs(d), np.abs(m), n, h, bc)


def tol_factor(n):
    """Multiply-adds along one output's longest chain, generously: 20 Q (n+1)^2."""
    q = (3 * n + 2) // 2
    return 20 * q * (n + 1) ** 2


CASES = [(n, bc, grid) for n in (1, 2, 3, 4, 5) for bc, grid in (("dirichlet", (20, 18, 17)), ("periodic", (19, 22, 16)))]


@pytest.mark.parametrize("n,bc,grid", CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_varcoef_apply_matches_oracle(n, bc, grid, dt, monkeypatch):
    print("varcoef", n, bc, grid, dt, flush=True)
    shape = grid[::-1]
    h = (1 / 21, 1 / 19, 1 / 18)
    tau = 2e-3
    c = rounded(normal_field(shape, 30 + n), dt)
    d, m = coef_fields(shape, 40 + n, tau)
    d, m = rounded(d, dt), rounded(m, dt)
    ctx = tbs.Context(grid, n, h, tau, bc)
    y = torch.empty(shape, dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")
    ctx.apply_varcoef(dev(c, dt), dev(d, dt), dev(m, dt), y)
    ref = varcoef.apply(c, d, m, n, h, bc)
    scale = abs_scale(c, d, m, n, h, bc, monkeypatch)
    tol = tol_factor(n) * EPS[dt] * scale + (np.abs(ref) * EPS[dt] if dt == "f32" else 0.0)
    err = np.abs(host(y) - ref)
    assert np.all(err <= tol), (err.max(), (err / scale).max())


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_constant_coefficients_give_the_heat_operator(bc):
    # d = tau and m = 1 everywhere: the quadrature operator equals A (the Toeplitz-filter apply)
    grid, n, tau = (26, 20, 18), 3, 1e-3
    h = (1 / 27, 1 / 21, 1 / 19)
    shape = grid[::-1]
    c = normal_field(shape, 5)
    ctx = tbs.Context(grid, n, h, tau, bc)
    y = torch.empty(shape, dtype=torch.float64, device="cuda")
    ctx.apply_varcoef(dev(c), dev(np.full(shape, tau)), dev(np.ones(shape)), y)
    ya = torch.empty_like(y)
    ctx.apply(dev(c), ya)
    ref = op.apply(c, n, h, tau, bc)
    assert np.max(np.abs(host(y) - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(host(y) - host(ya))) <= 1e-12 * np.max(np.abs(ref))


def test_varcoef_is_bitwise_reproducible():
    grid, n, tau = (70, 40, 36), 3, 1e-3
    h = (1 / 71, 1 / 41, 1 / 37)
    shape = grid[::-1]
    c = dev(normal_field(shape, 8), "f32")
    d, m = coef_fields(shape, 9, tau)
    d, m = dev(d, "f32"), dev(m, "f32")
    ctx = tbs.Context(grid, n, h, tau, "dirichlet")
    y1, y2 = torch.empty_like(c), torch.empty_like(c)
    ctx.apply_varcoef(c, d, m, y1)
    ctx.apply_varcoef(c, d, m, y2)
    assert torch.equal(y1, y2)


def test_varcoef_928_sampled(monkeypatch):
    # 928^3 cubic Dirichlet in FP32 (the size of the timed apply); each sampled output depends on
    # u within n of it and on d, m within n of it, so the oracle runs on that (2n+1)^3 block
    # (u zero-filled, d and m clamped to the grid beyond the box faces)
    N, n, tau = 928, 3, 1e-5
    h = (1 / 929,) * 3
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    c = torch.randn((N, N, N), generator=g, device="cuda", dtype=torch.float32)
    d = tau * (1.0 + 0.5 * torch.tanh(torch.randn((N, N, N), generator=g, device="cuda", dtype=torch.float32)))
    m = 1.0 + 0.5 * torch.tanh(torch.randn((N, N, N), generator=g, device="cuda", dtype=torch.float32))
    ctx = tbs.Context((N, N, N), n, h, tau, "dirichlet")
    y = torch.empty_like(c)
    ctx.apply_varcoef(c, d, m, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    pts = [tuple(rng.integers(0, N, 3)) for _ in range(60)]
    pts += [(0, 0, 0), (1, 2, 3), (N - 1, N - 1, N - 1), (N - 2, 5, 57), (400, 15, 16), (300, 58, 59), (7, N - 3, 116)]
    off = np.arange(-n, n + 1)
    for k, j, i in pts:
        zz, yy, xx = np.meshgrid(k + off, j + off, i + off, indexing="ij")
        inside = (zz >= 0) & (zz < N) & (yy >= 0) & (yy < N) & (xx >= 0) & (xx < N)
        zc, yc, xc = (torch.from_numpy(np.clip(a, 0, N - 1)).cuda() for a in (zz, yy, xx))
        cb = np.where(inside, c[zc, yc, xc].double().cpu().numpy(), 0.0)
        db = d[zc, yc, xc].double().cpu().numpy()
        mb = m[zc, yc, xc].double().cpu().numpy()
        ref = varcoef.apply(cb, db, mb, n, h, "dirichlet")[n, n, n]
        sc = abs_scale(cb, db, mb, n, h, "dirichlet", monkeypatch)[n, n, n]
        got = float(y[k, j, i])
        assert abs(got - ref) <= tol_factor(n) * EPS["f32"] * sc + abs(ref) * EPS["f32"], ((k, j, i), got, ref)
