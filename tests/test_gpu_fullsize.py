"""Full-size parity (928^3 Dirichlet cubic, 1024 x 512 x 256 periodic n = 2, 3, 5) on sampled
outputs: the oracle evaluates each sampled point from its (2n+1)^3 neighbourhood, which the
device input holds (gathered with zero fill / wrap-around)."""
import numpy as np
import pytest

from oracle import operator as op
from tests.gpu_util import op_tolerance
import workloads

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")
torch = pytest.importorskip("torch")


def sample_points(grid, count, seed, ty=32):
    """Random points plus faces, edges, corners and tile / chunk boundaries."""
    Nx, Ny, Nz = grid
    rng = np.random.default_rng(seed)
    pts = [rng.integers(0, N, count) for N in (Nz, Ny, Nx)]
    pts = np.stack(pts, axis=1)
    special = []
    for z in (0, 1, 2, 3, Nz // 2, Nz - 4, Nz - 3, Nz - 1):
        for y in (0, 2, ty - 1, ty, 16, Ny // 2, Ny - 1):
            for x in (0, 3, 63, 64, 65, Nx - 65, Nx - 64, Nx - 1):
                special.append((z, y, x))
    return np.concatenate([pts, np.array(special)])


def gather(t, pts, n, periodic):
    """Neighbourhoods [P, 2n+1, 2n+1, 2n+1] of the points, FP64 on the host."""
    Nz, Ny, Nx = t.shape
    off = torch.arange(-n, n + 1, device=t.device)
    p = torch.from_numpy(pts).to(t.device)
    z = p[:, 0, None, None, None] + off[None, :, None, None]
    y = p[:, 1, None, None, None] + off[None, None, :, None]
    x = p[:, 2, None, None, None] + off[None, None, None, :]
    z, y, x = torch.broadcast_tensors(z, y, x)
    if periodic:
        return t[z % Nz, y % Ny, x % Nx].to(torch.float64).cpu().numpy()
    ok = (z >= 0) & (z < Nz) & (y >= 0) & (y < Ny) & (x >= 0) & (x < Nx)
    vals = t[z.clamp(0, Nz - 1), y.clamp(0, Ny - 1), x.clamp(0, Nx - 1)]
    return torch.where(ok, vals, torch.zeros_like(vals)).to(torch.float64).cpu().numpy()


def oracle_points(blocks, n, h, tau, fn="apply"):
    """Centre value of the operator on each neighbourhood (the taps reach exactly the block)."""
    out, scale = np.empty(len(blocks)), np.empty(len(blocks))
    for i, blk in enumerate(blocks):
        if fn == "apply":
            out[i] = op.apply(blk, n, h, tau, "dirichlet")[n, n, n]
            scale[i] = op.abs_apply(blk, n, h, tau, "dirichlet")[n, n, n]
        else:
            out[i] = op.mass_apply(blk, n, "dirichlet")[n, n, n]
            scale[i] = op.mass_apply(np.abs(blk), n, "dirichlet")[n, n, n]
    return out, scale


@pytest.fixture(scope="module")
def field928():
    w = workloads.HEAT_928_DIRICHLET
    u = workloads.gaussian_sum(w.grid, w.bc, w.h, workloads.initial_field_gaussians(w), xp=torch,
                               device="cuda", dtype=torch.float64)
    g = torch.Generator(device="cuda")
    g.manual_seed(928)
    u += 0.1 * torch.randn(u.shape, generator=g, device="cuda", dtype=torch.float64)
    ctx = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc)
    ctx.ensure_workspace(tbs.PREC_MIXED)
    return w, u, ctx


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_apply_928_sampled(field928, dt):
    w, u, ctx = field928
    td = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
    src = u.to(td)
    y = torch.empty(u.shape, dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")
    ctx.apply(src, y)
    pts = sample_points(w.grid, 1500, 1)
    blocks = gather(src, pts, w.degree, False)
    ref, scale = oracle_points(blocks, w.degree, w.h, w.tau)
    got = y[tuple(torch.from_numpy(pts.T).cuda())].to(torch.float64).cpu().numpy()
    comp = "f64" if dt == "f64" else "f32"
    tol = op_tolerance(w.degree, comp, scale) + (np.abs(ref) * 2.0 ** -24 if comp == "f32" else 0)
    assert np.all(np.abs(got - ref) <= tol)
    del y


def test_rhs_928_sampled(field928):
    w, u, ctx = field928
    b = torch.empty_like(u)
    ctx.rhs(u, None, b)
    pts = sample_points(w.grid, 1000, 2, ty=16)
    ref, scale = oracle_points(gather(u, pts, w.degree, False), w.degree, w.h, w.tau, fn="mass")
    got = b[tuple(torch.from_numpy(pts.T).cuda())].cpu().numpy()
    assert np.all(np.abs(got - ref) <= op_tolerance(w.degree, "f64", scale))


def test_refined_step_928_sampled_residual(field928):
    w, u, ctx = field928
    un = torch.empty_like(u)
    st = ctx.timestep(u, None, un, tbs.PREC_MIXED, w.rtol, 2000)
    assert st["converged"] and st["rel_res_fp64"] <= w.rtol
    # the oracle's residual at sampled points: r_i = (M u)_i - (A u_next)_i
    pts = sample_points(w.grid, 1500, 3, ty=16)
    bi, _ = oracle_points(gather(u, pts, w.degree, False), w.degree, w.h, w.tau, fn="mass")
    ai, sc = oracle_points(gather(un, pts, w.degree, False), w.degree, w.h, w.tau)
    r = bi - ai
    # sampled residual RMS consistent with the device's global FP64 residual (generous factor)
    assert np.sqrt(np.mean(r * r)) <= 20 * w.rtol * np.sqrt(np.mean(bi * bi)) + 1e-14 * np.max(sc)
    del un


@pytest.mark.parametrize("n", [2, 3, 5])
def test_apply_periodic_1024x512x256_sampled(n):
    w = workloads.HEAT_1024x512x256_PERIODIC
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    u = torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=torch.float32)
    ctx = tbs.Context(w.grid, n, w.h, w.tau, w.bc)
    ctx.ensure_workspace(-1)
    y = torch.empty_like(u)
    ctx.apply(u, y)
    pts = sample_points(w.grid, 1500, 5 + n)
    blocks = gather(u, pts, n, True)
    ref, scale = np.empty(len(pts)), np.empty(len(pts))
    for i, blk in enumerate(blocks):
        # the neighbourhood already holds the wrapped values: evaluate as a truncated block
        ref[i] = op.apply(blk, n, w.h, w.tau, "dirichlet")[n, n, n]
        scale[i] = op.abs_apply(blk, n, w.h, w.tau, "dirichlet")[n, n, n]
    got = y[tuple(torch.from_numpy(pts.T).cuda())].to(torch.float64).cpu().numpy()
    tol = op_tolerance(n, "f32", scale) + np.abs(ref) * 2.0 ** -24
    assert np.all(np.abs(got - ref) <= tol)


def test_periodic_1024x512x256_refined_steps_converge_and_conserve():
    # two refined FP32 steps of the cubic periodic workload: FP64 residual <= rtol and, with no
    # source on a periodic grid, sum u is conserved up to the residual (|sum r| <= sqrt(N) ||r||)
    w = workloads.HEAT_1024x512x256_PERIODIC
    g = torch.Generator(device="cuda")
    g.manual_seed(w.seed)
    u = torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=torch.float64)
    ctx = tbs.Context(w.grid, 3, w.h, w.tau, w.bc)
    ctx.ensure_workspace(tbs.PREC_MIXED)
    t = torch.empty_like(u)
    for _ in range(w.smooth_passes):
        ctx.rhs(u, None, t)
        u, t = t, u
    s0, a0 = float(u.sum()), float(u.abs().sum())
    for _ in range(2):
        st = ctx.timestep(u, None, t, tbs.PREC_MIXED, w.rtol, 2000)
        assert st["converged"] and st["rel_res_fp64"] <= w.rtol
        u, t = t, u
    assert abs(float(u.sum()) - s0) <= 1e-7 * a0
