"""Parity of the direct and indirect B-spline transforms with the FP64 oracle."""
import numpy as np
import pytest

from oracle import transforms as tr
from tests.gpu_util import dev, host, rounded
from workloads import normal_field

pytestmark = pytest.mark.gpu
tbs = pytest.importorskip("paper_1904_03057_amd")

CASES = [(2, (37, 11, 13), "periodic"), (3, (64, 33, 18), "dirichlet"), (3, (40, 24, 20), "periodic"),
         (4, (45, 19, 21), "dirichlet"), (5, (70, 22, 24), "periodic"), (5, (29, 30, 17), "dirichlet")]


def _abs_eval(c, n, bc):
    return tr.evaluate(np.abs(c), n, bc)


@pytest.mark.parametrize("n,grid,bc", CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_eval_matches_oracle(n, grid, bc, dt):
    c = normal_field(grid[::-1], 40 + n)
    if dt == "f32":
        c = rounded(c, "f32")
    t = tbs.Transform(grid, n, bc)
    t.ensure_workspace(-1)
    s = dev(np.zeros(grid[::-1]), dt)
    t.eval(dev(c, dt), s)
    ref = tr.evaluate(c, n, bc)
    scale = _abs_eval(c, n, bc)
    eps = 2.0 ** -52 if dt == "f64" else 2.0 ** -23
    # three passes of at most 5 taps: a few roundings per output, relative to the absolute sum
    assert np.all(np.abs(host(s) - ref) <= 12 * eps * scale)


@pytest.mark.parametrize("n,grid,bc", CASES)
def test_interp_matches_oracle_and_round_trips(n, grid, bc):
    s = normal_field(grid[::-1], 50 + n)
    t = tbs.Transform(grid, n, bc)
    sd = dev(s)
    c = sd.clone()  # start from the samples
    it, rel = t.interp(sd, c, rtol=1e-13, max_iter=500)
    # CG stops on its recursive residual; the true FP64 residual recomputed at exit may sit a
    # little above rtol this close to FP64 precision
    assert rel <= 1.1e-13 and it > 0
    ref = tr.interpolate(s, n, bc)
    # error <= kappa(E) * rtol, kappa(E) <= (1 / Bhat(pi))^3 <= 7.5^3
    assert np.linalg.norm(host(c) - ref) <= 450 * 1.2e-13 * np.linalg.norm(ref)
    back = dev(np.zeros(grid[::-1]))
    t.eval(c, back)
    assert np.linalg.norm(host(back) - s) <= 2e-13 * np.linalg.norm(s)


def test_interp_of_sampled_spline_recovers_coefficients_at_928_sized_plane():
    # full x-y plane of the 928^3 workload with a thin z extent: coefficients -> samples -> back
    grid = (928, 928, 12)
    c0 = normal_field(grid[::-1], 77)
    t = tbs.Transform(grid, 3, "dirichlet")
    s = dev(np.zeros(grid[::-1]))
    t.eval(dev(c0), s)
    c = s.clone()
    it, rel = t.interp(s, c, rtol=1e-12, max_iter=500)
    assert rel <= 1.1e-12
    assert np.linalg.norm(host(c) - c0) <= 27 * 1.2e-12 * np.linalg.norm(c0)
