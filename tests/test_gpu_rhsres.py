"""The fused right-hand side and first residual of a source-free refined step (one pass over u^k
forming b = M u^k and b - A u^k) against the separate rhs and residual kernels: the steps agree bit
for bit, and their answers pass the oracle's residual test.  Also the sweeps' convergence checks
(norms only when a check is expected to pass) at tolerances down to 1e-12, and that no step reads
workspace contents it did not write (the inner correction starts as zero without a fill)."""
import numpy as np
import pytest

from oracle import operator as op, solvers
from tests.gpu_util import dev, host
from workloads import normal_field

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")


@pytest.mark.parametrize("n,grid,bc", [(1, (23, 17, 9), "dirichlet"), (3, (70, 22, 20), "dirichlet"),
                                       (3, (64, 24, 18), "periodic"), (5, (45, 19, 21), "periodic"),
                                       (2, (37, 50, 13), "dirichlet")])
@pytest.mark.parametrize("prec", ["MIXED", "MIXED_BF16"])
def test_fused_rhs_and_residual_step_equals_separate_kernels(n, grid, bc, prec):
    h = tuple(1.0 / N for N in grid)
    tau, rtol = 2e-3, 1e-9
    P = getattr(tbs, "PREC_" + prec)
    u = normal_field(grid[::-1], 60 + n)
    outs, stats = [], []
    for fused in (1, 0):
        ctx = tbs.Context(grid, n, h, tau, bc)
        ctx.set_opts(fused_rhs=fused)
        ctx.ensure_workspace(P)
        un = dev(np.zeros(grid[::-1]))
        st = ctx.timestep(dev(u), None, un, P, rtol, 2000)
        assert st["converged"], st
        outs.append(host(un))
        stats.append(st)
    assert np.array_equal(outs[0], outs[1])
    assert stats[0]["iters"] == stats[1]["iters"] and stats[0]["sweeps"] == stats[1]["sweeps"]
    assert stats[0]["rel_res0"] == stats[1]["rel_res0"]
    # the oracle's FP64 residual of the answer
    b = op.rhs(u, None, n, tau, bc)
    assert solvers.rel_residual(lambda v: op.apply(v, n, h, tau, bc), b, outs[0]) <= rtol * 1.01


def test_fused_rhs_is_not_taken_with_a_source():
    # with q the step takes the rhs and residual kernels; q = 0 gives the same answer as q = None
    grid, n, bc = (40, 24, 18), 3, "dirichlet"
    h = tuple(1.0 / N for N in grid)
    u = normal_field(grid[::-1], 7)
    ctx = tbs.Context(grid, n, h, 1e-3, bc)
    ctx.ensure_workspace(tbs.PREC_MIXED)
    a, b = dev(np.zeros(grid[::-1])), dev(np.zeros(grid[::-1]))
    s1 = ctx.timestep(dev(u), None, a, tbs.PREC_MIXED, 1e-9, 2000)
    s2 = ctx.timestep(dev(u), dev(np.zeros(grid[::-1])), b, tbs.PREC_MIXED, 1e-9, 2000)
    assert np.array_equal(host(a), host(b)) and s1["iters"] == s2["iters"]


@pytest.mark.parametrize("rtol", [1e-8, 1e-10, 1e-12])
@pytest.mark.parametrize("n,grid,bc", [(3, (70, 22, 20), "dirichlet"), (2, (64, 24, 18), "periodic")])
def test_refined_steps_convergence_checks(n, grid, bc, rtol):
    # each sweep's check of the refined step: a check expected to pass forms only the norms and
    # stores the FP32 residual only if it fails; whichever way it goes, every answer meets rtol in
    # the oracle's FP64 residual
    print("check", n, grid, bc, rtol, flush=True)
    h = tuple(1.0 / N for N in grid)
    tau = 2e-3
    ctx = tbs.Context(grid, n, h, tau, bc)
    ctx.ensure_workspace(tbs.PREC_MIXED)
    u = normal_field(grid[::-1], 90 + n)
    ua, ub = dev(u), dev(np.zeros(grid[::-1]))
    for _ in range(3):
        st = ctx.timestep(ua, None, ub, tbs.PREC_MIXED, rtol, 4000)
        assert st["converged"] and st["rel_res_fp64"] <= rtol, st
        b = op.rhs(host(ua), None, n, tau, bc)
        assert solvers.rel_residual(lambda v: op.apply(v, n, h, tau, bc), b, host(ub)) <= rtol * 1.01
        ua, ub = ub, ua


@pytest.mark.parametrize("prec", ["MIXED", "MIXED_BF16"])
@pytest.mark.parametrize("n,grid,bc", [(3, (70, 22, 20), "dirichlet"), (1, (23, 17, 9), "periodic")])
def test_refined_steps_read_no_stale_workspace(n, grid, bc, prec):
    # the inner solve's correction d starts as zero without being filled (its first update writes
    # it, the refinement update takes it as zero until then): steps on a workspace filled with NaN
    # bytes before every step equal the steps on a fresh one bit for bit
    import torch
    print("stale", n, grid, bc, prec, flush=True)
    h = tuple(1.0 / N for N in grid)
    P = getattr(tbs, "PREC_" + prec)
    u = normal_field(grid[::-1], 120 + n)
    outs = []
    for poison in (False, True):
        ctx = tbs.Context(grid, n, h, 2e-3, bc)
        ws = ctx.ensure_workspace(P)
        ua, ub = dev(u), dev(np.zeros(grid[::-1]))
        res = []
        for rtol in (1e-9, 1e-3, 1e-12):  # 1e-3: a short inner solve, possibly with no x update
            if poison:
                ws.fill_(0xFF)
                torch.cuda.synchronize()
            st = ctx.timestep(ua, None, ub, P, rtol, 4000)
            assert st["converged"], st
            res.append((host(ub), st["iters"], st["sweeps"]))
            ua, ub = ub, ua
        outs.append(res)
    for (a, ia, sa), (b, ib, sb) in zip(*outs):
        assert np.array_equal(a, b) and np.all(np.isfinite(a)) and ia == ib and sa == sb
