"""A CG solve captured into a HIP graph through the C ABI (poll_every = 0: tbs_cg_begin and
tbs_cg_step enqueue their kernels and never wait on the host) and replayed on new right-hand sides:
every replay equals the eager solve bit for bit and follows the oracle's Hestenes-Stiefel CG."""
import numpy as np
import pytest

from oracle import operator as op, solvers
from tests.gpu_util import dev, host, rounded
from workloads import normal_field

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec,fused", [("f64", 1), ("f64", 0), ("f32", 1), ("f32", 0)])
def test_cg_solve_captured_in_a_graph_replays_like_eager(prec, fused):
    grid, n, bc, k = (40, 24, 18), 3, "dirichlet", 9
    h, tau = tuple(1.0 / N for N in grid), 2e-3
    P = tbs.PREC_FP64 if prec == "f64" else tbs.PREC_FP32
    tdt = torch.float64 if prec == "f64" else torch.float32
    side = torch.cuda.Stream()
    cap = tbs.Context(grid, n, h, tau, bc, stream=side)
    cap.set_opts(poll_every=0, fused_cg=fused)
    cap.ensure_workspace(P)
    eager = tbs.Context(grid, n, h, tau, bc)
    eager.set_opts(fused_cg=fused)
    eager.ensure_workspace(P)
    b = torch.zeros(grid[::-1], dtype=tdt, device="cuda")
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        cap.cg_begin(b, x, 0.0)
        cap.cg_step(k, sync=False)
    torch.cuda.synchronize()
    A = lambda v: op.apply(v, n, h, tau, bc)
    for seed in (1, 2, 3):
        bb = rounded(normal_field(grid[::-1], 40 + seed), prec)
        b.copy_(dev(bb, prec))
        x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = host(x)
        # eager work between the replays: the same solve on another context and stream
        xe = dev(np.zeros(grid[::-1]), prec)
        eager.cg_begin(dev(bb, prec), xe, 0.0)
        rel, it = eager.cg_step(k)
        assert it == k
        assert np.array_equal(got, host(xe)), seed
        xr, _, _ = solvers.cg(A, bb, np.zeros_like(bb), 0.0, 100, fixed_iters=k)
        tol = 1e-10 if prec == "f64" else 1e-4
        assert np.linalg.norm(got - xr) <= tol * np.linalg.norm(xr), seed
