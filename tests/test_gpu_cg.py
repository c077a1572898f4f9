"""Parity of the fused CG, refinement and implicit time step with the FP64 oracle."""
import numpy as np
import pytest

from oracle import exact, operator as op, solvers
from tests.gpu_util import dev, host, rounded
from workloads import HEAT_32_PERIODIC, normal_field, sine_modes

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")


def _ctx(grid, n, h, tau, bc, prec):
    c = tbs.Context(grid, n, h, tau, bc)
    c.ensure_workspace(prec)
    return c


def config1_fields():
    w = HEAT_32_PERIODIC
    shape = w.grid[::-1]
    u0 = op.mass_apply(op.mass_apply(normal_field(shape, w.seed), w.degree, w.bc), w.degree, w.bc)
    u0 = u0 + sine_modes(w.grid, w.h, w.seed + 1)
    return w, u0


@pytest.mark.parametrize("bc,grid", [("dirichlet", (40, 24, 18)), ("periodic", (32, 20, 16))])
@pytest.mark.parametrize("k", [1, 3, 12])
@pytest.mark.parametrize("fused", [1, 0])
def test_cg_iterate_parity_fp64(bc, grid, k, fused):
    # both FP64 iteration forms (one kernel with the r.r prediction, two kernels) against the
    # oracle's Hestenes-Stiefel iterates
    n, h, tau = 3, (1 / 40, 1 / 24, 1 / 18), 2e-3
    b = normal_field(grid[::-1], 11)
    x0 = normal_field(grid[::-1], 12) * 0.1
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP64)
    ctx.set_opts(fused_cg=fused)
    ctx.ensure_workspace(tbs.PREC_FP64)
    x = dev(x0)
    ctx.cg_begin(dev(b), x, 0.0)
    rel, it = ctx.cg_step(k)
    A = lambda v: op.apply(v, n, h, tau, bc)
    xr, _, hist = solvers.cg(A, b, x0, 0.0, 100, fixed_iters=k)
    assert it == k
    assert np.linalg.norm(host(x) - xr) <= 1e-10 * np.linalg.norm(xr)
    assert abs(rel - hist[-1]) <= 1e-8 * hist[-1]


@pytest.mark.parametrize("fused", [1, 0])
def test_cg_step_continuation_bitwise(fused):
    grid, n, h, tau, bc = (33, 21, 17), 2, (0.03, 0.05, 0.06), 1e-3, "periodic"
    b = dev(normal_field(grid[::-1], 1))
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP64)
    ctx.set_opts(fused_cg=fused)
    ctx.ensure_workspace(tbs.PREC_FP64)
    x1 = dev(np.zeros(grid[::-1]))
    ctx.cg_begin(b, x1, 0.0)
    ctx.cg_step(10)
    x2 = dev(np.zeros(grid[::-1]))
    ctx.cg_begin(b, x2, 0.0)
    ctx.cg_step(4)
    ctx.cg_step(6)
    assert np.array_equal(host(x1), host(x2))


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("bc,grid", [("dirichlet", (48, 20, 22)), ("periodic", (64, 24, 20))])
def test_cg_fp32_iterates_close_to_oracle(fused, bc, grid):
    # both FP32 iteration forms (one kernel with the r.r prediction, two kernels) follow the oracle's
    # Hestenes-Stiefel iterates and residual history to FP32 accuracy
    n, tau = 3, 1e-3
    h = tuple(1.0 / N for N in grid)
    b = rounded(normal_field(grid[::-1], 2), "f32")
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP32)
    ctx.set_opts(fused_cg=fused)
    ctx.ensure_workspace(tbs.PREC_FP32)
    x = dev(np.zeros(grid[::-1]), "f32")
    ctx.cg_begin(dev(b, "f32"), x, 0.0)
    rel, it = ctx.cg_step(8)
    xr, _, hist = solvers.cg(lambda v: op.apply(v, n, h, tau, bc), b, np.zeros_like(b), 0.0, 100, fixed_iters=8)
    assert it == 8
    assert np.linalg.norm(host(x) - xr) <= 1e-4 * np.linalg.norm(xr)
    assert abs(rel - hist[-1]) <= 1e-3 * hist[-1], (rel, hist[-1])


@pytest.mark.parametrize("n,grid,bc", [(1, (23, 17, 9), "dirichlet"), (2, (37, 11, 13), "periodic"),
                                       (4, (45, 19, 21), "dirichlet"), (5, (70, 22, 24), "periodic")])
def test_cg_fp32_one_kernel_other_degrees(n, grid, bc):
    # ragged grids (not multiples of the tile or vector width) and the other basis degrees
    tau = 2e-3
    h = tuple(1.0 / N for N in grid)
    b = rounded(normal_field(grid[::-1], 6 + n), "f32")
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP32)
    x = dev(np.zeros(grid[::-1]), "f32")
    ctx.cg_begin(dev(b, "f32"), x, 0.0)
    rel, it = ctx.cg_step(6)
    xr, _, hist = solvers.cg(lambda v: op.apply(v, n, h, tau, bc), b, np.zeros_like(b), 0.0, 100, fixed_iters=6)
    assert it == 6
    assert np.linalg.norm(host(x) - xr) <= 1e-4 * np.linalg.norm(xr)
    assert abs(rel - hist[-1]) <= 1e-3 * hist[-1], (rel, hist[-1])


@pytest.mark.parametrize("n", [1, 3, 5])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("dt,fused", [("f64", 1), ("f64", 0), ("f32", 1), ("f32", 0)])
def test_cg_on_the_smallest_grid(n, bc, dt, fused):
    # every axis at the 2n+1 minimum: one partial tile, one z-chunk shorter than its halo; the
    # iterates of both forms against the oracle's Hestenes-Stiefel CG
    N = 2 * n + 1
    grid, tau, k = (N, N, N), 1e-2, 4
    h = (1.0 / N,) * 3
    P = tbs.PREC_FP64 if dt == "f64" else tbs.PREC_FP32
    ctx = _ctx(grid, n, h, tau, bc, P)
    ctx.set_opts(fused_cg=fused)
    ctx.ensure_workspace(P)
    b = rounded(normal_field(grid[::-1], 50 + n), dt)
    x = dev(np.zeros(grid[::-1]), dt)
    ctx.cg_begin(dev(b, dt), x, 0.0)
    rel, it = ctx.cg_step(k)
    xr, _, hist = solvers.cg(lambda v: op.apply(v, n, h, tau, bc), b, np.zeros_like(b), 0.0, 100, fixed_iters=k)
    assert it == k
    tol = 1e-10 if dt == "f64" else 1e-4
    assert np.linalg.norm(host(x) - xr) <= tol * np.linalg.norm(xr)


@pytest.mark.parametrize("split", [(4, 5), (3, 6), (1, 1, 7), (2, 2, 2, 3)])
def test_cg_fp32_one_kernel_continuation_bitwise(split):
    # r, p and q alternate between two arrays, and x takes its updates two at a time (flushed at the
    # end of each call, one or two pending): splitting the iterations over calls changes nothing
    grid, n, h, tau, bc = (40, 18, 20), 3, (1 / 40, 1 / 18, 1 / 20), 1e-3, "dirichlet"
    b = dev(rounded(normal_field(grid[::-1], 5), "f32"), "f32")
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP32)
    x1 = dev(np.zeros(grid[::-1]), "f32")
    ctx.cg_begin(b, x1, 0.0)
    ctx.cg_step(sum(split))
    x2 = dev(np.zeros(grid[::-1]), "f32")
    ctx.cg_begin(b, x2, 0.0)
    for k in split:
        ctx.cg_step(k)
    assert np.array_equal(host(x1), host(x2))


@pytest.mark.parametrize("k", [1, 2, 3, 6, 7])
def test_cg_fp32_one_kernel_x_after_k_iterations(k):
    # the iterate after k one-kernel iterations (0, 1 or 2 updates pending at the end) against the
    # oracle's Hestenes-Stiefel iterate, and against the two-kernel form, which updates x every
    # iteration: both apply the same FP32 updates, so their x agree to FP32 rounding of the operator
    grid, n, bc = (48, 20, 22), 3, "dirichlet"
    tau, h = 1e-3, tuple(1.0 / N for N in grid)
    b = rounded(normal_field(grid[::-1], 3), "f32")
    xs = []
    for fused in (1, 0):
        ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP32)
        ctx.set_opts(fused_cg=fused)
        ctx.ensure_workspace(tbs.PREC_FP32)
        x = dev(np.zeros(grid[::-1]), "f32")
        ctx.cg_begin(dev(b, "f32"), x, 0.0)
        assert ctx.cg_step(k)[1] == k
        xs.append(host(x))
    xr, _, _ = solvers.cg(lambda v: op.apply(v, n, h, tau, bc), b, np.zeros_like(b), 0.0, 100, fixed_iters=k)
    assert np.linalg.norm(xs[0] - xr) <= 1e-4 * np.linalg.norm(xr)
    assert np.linalg.norm(xs[0] - xs[1]) <= 1e-4 * np.linalg.norm(xr)


@pytest.mark.parametrize("fused", [1, 0])
def test_config1_fp64_step_matches_fft_exact_and_conserves(fused):
    w, u0 = config1_fields()
    ctx = _ctx(w.grid, w.degree, w.h, w.tau, w.bc, tbs.PREC_FP64)
    ctx.set_opts(fused_cg=fused)
    ctx.ensure_workspace(tbs.PREC_FP64)
    un = dev(np.zeros(u0.shape))
    st = ctx.timestep(dev(u0), None, un, tbs.PREC_FP64, w.rtol, 500)
    assert st["converged"]
    u1 = host(un)
    A = lambda v: op.apply(v, w.degree, w.h, w.tau, w.bc)
    b = op.rhs(u0, None, w.degree, w.tau, w.bc)
    # (iii) the oracle's FP64 residual of the GPU answer
    assert solvers.rel_residual(A, b, u1) <= w.rtol * 1.01
    assert abs(st["rel_res_fp64"] - solvers.rel_residual(A, b, u1)) <= 1e-3 * w.rtol
    # (ii) iterate parity: the oracle's CG with the GPU's iteration count
    xr, _, _ = solvers.cg(A, b, u0, 0.0, 500, fixed_iters=st["iters"])
    assert np.linalg.norm(u1 - xr) <= 1e-10 * np.linalg.norm(xr)
    _, it_ref, _ = solvers.cg(A, b, u0, w.rtol, 500)
    assert abs(it_ref - st["iters"]) <= 1
    # error against the exact FFT step is bounded by kappa * rtol
    xs = exact.step(u0, None, w.degree, w.h, w.tau, w.bc)
    kappa = exact.condition_number(w.grid, w.degree, w.h, w.tau, w.bc)
    assert np.linalg.norm(u1 - xs) / np.linalg.norm(xs) <= kappa * w.rtol
    # conservation: sum u^{k+1} = sum u^k (f = 0)
    assert abs(u1.sum() - u0.sum()) <= 1e-9 * np.abs(u0).sum()


def test_config1_tight_tolerance_reaches_1e10_error():
    w, u0 = config1_fields()
    ctx = _ctx(w.grid, w.degree, w.h, w.tau, w.bc, tbs.PREC_FP64)
    un = dev(np.zeros(u0.shape))
    st = ctx.timestep(dev(u0), None, un, tbs.PREC_FP64, 1e-13, 500)
    xs = exact.step(u0, None, w.degree, w.h, w.tau, w.bc)
    assert np.linalg.norm(host(un) - xs) / np.linalg.norm(xs) <= 1e-10


@pytest.mark.parametrize("prec,fused", [("MIXED", 1), ("MIXED_BF16", 1), ("MIXED", 0), ("MIXED_BF16", 0),
                                        ("FP64", 1)])
def test_dirichlet_step_refined_matches_fdm_exact(prec, fused):
    grid, n, tau = (48, 40, 36), 3, 1e-4
    h = tuple(1.0 / (N + 1) for N in grid)
    u0 = normal_field(grid[::-1], 21)
    q = normal_field(grid[::-1], 22) * 10
    p = getattr(tbs, "PREC_" + prec)
    ctx = _ctx(grid, n, h, tau, "dirichlet", p)
    ctx.set_opts(fused_cg=fused)
    un = dev(np.zeros(grid[::-1]))
    st = ctx.timestep(dev(u0), dev(q), un, p, 1e-8, 2000)
    assert st["converged"], st
    A = lambda v: op.apply(v, n, h, tau, "dirichlet")
    b = op.rhs(u0, q, n, tau, "dirichlet")
    u1 = host(un)
    rr = solvers.rel_residual(A, b, u1)
    assert rr <= 1e-8 * 1.01, (rr, st)
    xs = exact.step(u0, q, n, h, tau, "dirichlet")
    kappa = exact.condition_number(grid, n, h, tau, "dirichlet")
    assert np.linalg.norm(u1 - xs) / np.linalg.norm(xs) <= kappa * 1e-8
    if prec != "FP64":
        assert st["sweeps"] >= 1


def test_raw_fp32_step_config_like_within_1e5():
    # smooth Gaussian-sum field and source at the diffusion number tau/h^2 = 6.6 of the 256^3 workload
    from workloads import gaussian_params, gaussian_sum
    grid, n = (64, 64, 64), 3
    h = tuple(1.0 / (N + 1) for N in grid)
    tau = 6.6 * h[0] ** 2
    u0 = gaussian_sum(grid, "dirichlet", h, gaussian_params(4, 16, 0.05, 0.1, 1.0, 0.2, 0.8))
    q = gaussian_sum(grid, "dirichlet", h, gaussian_params(5, 2, 0.05, 0.15, 10.0, 0.2, 0.8))
    ctx = _ctx(grid, n, h, tau, "dirichlet", tbs.PREC_FP32)
    un = dev(np.zeros(grid[::-1]))
    st = ctx.timestep(dev(u0), dev(q), un, tbs.PREC_FP32, 1e-6, 500)
    xs = exact.step(u0, q, n, h, tau, "dirichlet")
    err = np.linalg.norm(host(un) - xs) / np.linalg.norm(xs)
    assert err <= 1e-5, err
    assert st["rel_res_fp64"] <= 1e-5


def test_raw_fp32_rough_field_within_condition_bound():
    # rough N(0,1) data at a small diffusion number: A is close to the ill-conditioned mass matrix,
    # so only the kappa * eps_32 bound holds for raw FP32 (refinement is what recovers accuracy)
    grid, n, tau = (40, 40, 40), 3, 1e-4
    h = tuple(1.0 / (N + 1) for N in grid)
    u0 = normal_field(grid[::-1], 31)
    ctx = _ctx(grid, n, h, tau, "dirichlet", tbs.PREC_FP32)
    un = dev(np.zeros(grid[::-1]))
    ctx.timestep(dev(u0), None, un, tbs.PREC_FP32, 1e-6, 500)
    xs = exact.step(u0, None, n, h, tau, "dirichlet")
    err = np.linalg.norm(host(un) - xs) / np.linalg.norm(xs)
    kappa = exact.condition_number(grid, n, h, tau, "dirichlet")
    assert err <= 4 * kappa * 2.0 ** -24, (err, kappa)
    ctx.ensure_workspace(tbs.PREC_MIXED)
    st = ctx.timestep(dev(u0), None, un, tbs.PREC_MIXED, 1e-12, 2000)
    assert np.linalg.norm(host(un) - xs) / np.linalg.norm(xs) <= kappa * 1e-12 * 2


def test_zero_rhs_and_iteration_limit_and_breakdown():
    grid, n, h, tau, bc = (20, 18, 16), 2, (0.05, 0.05, 0.05), 1e-3, "dirichlet"
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_FP64)  # the FP64 layout is the largest
    z = dev(np.zeros(grid[::-1]))
    un = dev(np.ones(grid[::-1]))
    st = ctx.timestep(z, None, un, tbs.PREC_FP64, 1e-10, 100)
    assert st["converged"] and st["iters"] == 0 and np.all(host(un) == 0)
    u0 = dev(normal_field(grid[::-1], 5))
    st = ctx.timestep(u0, None, un, tbs.PREC_FP64, 1e-14, 1)
    assert not st["converged"] and st["iters"] == 1
    bad = normal_field(grid[::-1], 6)
    bad[3, 4, 5] = np.nan
    for prec in (tbs.PREC_FP64, tbs.PREC_MIXED):
        with pytest.raises(tbs.TbsError) as e:
            ctx.timestep(dev(bad), None, un, prec, 1e-8, 100)
        assert e.value.code == tbs.E_BREAKDOWN


def test_timestep_bitwise_reproducible_and_resumable():
    grid, n, h, tau, bc = (36, 28, 20), 3, (1 / 37, 1 / 29, 1 / 21), 1e-4, "dirichlet"
    u0 = dev(normal_field(grid[::-1], 8))
    q = dev(normal_field(grid[::-1], 9))
    ctx = _ctx(grid, n, h, tau, bc, tbs.PREC_MIXED)

    def run(u, steps):
        a, b = u.clone(), dev(np.zeros(grid[::-1]))
        for _ in range(steps):
            ctx.timestep(a, q, b, tbs.PREC_MIXED, 1e-8, 500)
            a, b = b, a
        return a

    straight = host(run(u0, 4))
    half = run(u0, 2)
    ckpt = host(half)                # checkpoint: the state is the coefficient tensor
    resumed = host(run(dev(ckpt), 2))
    assert np.array_equal(straight, resumed)
    assert np.array_equal(straight, host(run(u0, 4)))


@pytest.mark.parametrize("prec", [tbs.PREC_FP64, tbs.PREC_MIXED, tbs.PREC_MIXED_BF16])
@pytest.mark.parametrize("coarse", [0, 1])
def test_timestep_output_independent_of_prior_contents(prec, coarse):
    # u_next is output only: the step writes every entry whatever it held before (the refined
    # path forms u_next = u_prev + d on its first correction instead of copying u_prev first)
    grid, n, tau = (40, 26, 18), 3, 2e-3
    h = tuple(1.0 / (N + 1) for N in grid)
    u = dev(normal_field(grid[::-1], 21))
    ctx = tbs.Context(grid, n, h, tau, "dirichlet")
    ctx.set_opts(coarse_guess=coarse)
    ctx.ensure_workspace(prec)
    a = dev(np.zeros(grid[::-1]))
    b = dev(np.full(grid[::-1], np.nan))
    sa = ctx.timestep(u, None, a, prec, 1e-8, 2000)
    sb = ctx.timestep(u, None, b, prec, 1e-8, 2000)
    assert sa["converged"] and sb["converged"]
    assert np.array_equal(host(a), host(b))
    # a step that needs no correction returns its initial guess: u_prev itself, or the coarse guess
    c = dev(np.full(grid[::-1], np.nan))
    sc = ctx.timestep(u, None, c, prec, 10.0, 2000)
    assert sc["iters"] == 0 and np.all(np.isfinite(host(c)))
    if not sc["used_coarse_guess"]:
        assert np.array_equal(host(c), host(u))


@pytest.mark.parametrize("mag", [1e-36, 3e37])
def test_refinement_keeps_the_inner_residual_in_fp32_range(mag):
    # the refinement solves A d = r / s (s a power of two near the residual's RMS) whenever r's
    # elements would leave the normal FP32 range, and adds s d back in FP64: fields at 1e-36 and
    # 3e37 reach the oracle's exact step as fields of size one do
    grid, n, tau, rtol = (40, 24, 20), 3, 1e-3, 1e-10
    h = tuple(1.0 / (N + 1) for N in grid)
    u = op.mass_apply(normal_field(grid[::-1], 14), n, "dirichlet") * mag
    ctx = _ctx(grid, n, h, tau, "dirichlet", tbs.PREC_MIXED)
    un = dev(np.zeros(grid[::-1]))
    st = ctx.timestep(dev(u), None, un, tbs.PREC_MIXED, rtol, 2000)
    assert st["converged"], st
    b = op.rhs(u, None, n, tau, "dirichlet")
    got = host(un)
    assert np.linalg.norm(b - op.apply(got, n, h, tau, "dirichlet")) <= rtol * (1 + 1e-6) * np.linalg.norm(b)
    xs = exact.solve_dirichlet(b, n, h, tau)
    kappa = exact.condition_number(grid, n, h, tau, "dirichlet")
    assert np.linalg.norm(got - xs) <= kappa * rtol * np.linalg.norm(xs)
