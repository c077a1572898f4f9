"""Parity of the HIP operator kernels (apply, rhs, residual, dot, convert) with the FP64 oracle."""
import numpy as np
import pytest

from oracle import operator as op
from tests.gpu_util import dev, host, op_tolerance, rounded
from workloads import normal_field

pytestmark = pytest.mark.gpu

tbs = pytest.importorskip("paper_1904_03057_amd")

# shapes span several 64 x 16 tiles with ragged tails; tiny shapes hit the 2n+1 minimum
SHAPES = [(130, 37, 29), (64, 16, 20), (7, 7, 7), (33, 17, 9), (200, 5, 11)]


def _ctx(grid, n, h, tau, bc, zchunk=0):
    c = tbs.Context(grid, n, h, tau, bc)
    if zchunk:
        c.set_opts(zchunk=zchunk)
    c.ensure_workspace(-1)
    return c


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("shape_i", range(len(SHAPES)))
def test_apply_f64_matches_oracle(bc, n, shape_i):
    grid = SHAPES[shape_i]
    if min(grid) < 2 * n + 1:
        pytest.skip("grid below 2n+1")
    h, tau = (0.031, 0.047, 0.029), 2.3e-3
    u = normal_field(grid[::-1], 100 + n)
    ctx = _ctx(grid, n, h, tau, bc)
    y = dev(np.zeros(grid[::-1]))
    ctx.apply(dev(u), y)
    ref = op.apply(u, n, h, tau, bc)
    tol = op_tolerance(n, "f64", op.abs_apply(u, n, h, tau, bc))
    assert np.all(np.abs(host(y) - ref) <= tol)


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("n", [2, 3, 5])
@pytest.mark.parametrize("pair", [("f32", "f32"), ("bf16", "f32"), ("f32", "f64"), ("bf16", "f64")])
def test_apply_reduced_precision_on_rounded_inputs(bc, n, pair):
    din, dout = pair
    grid = (97, 35, 23)
    h, tau = (1 / 97, 1 / 35, 1 / 23), 1e-4
    u = rounded(normal_field(grid[::-1], 7), din)
    ctx = _ctx(grid, n, h, tau, bc)
    y = dev(np.zeros(grid[::-1]), dout)
    ctx.apply(dev(u, din), y)
    ref = op.apply(u, n, h, tau, bc)
    tol = op_tolerance(n, "f64" if dout == "f64" else "f32", op.abs_apply(u, n, h, tau, bc))
    if dout == "f32":
        tol = tol + np.abs(ref) * 2.0 ** -24  # final rounding of the stored result
    assert np.all(np.abs(host(y) - ref) <= tol)


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("n", [1, 3, 5])
def test_zchunk_and_repeat_bitwise_identical(bc, n):
    grid = (70, 40, 61)
    h, tau = (0.02, 0.03, 0.025), 1e-3
    u = dev(normal_field(grid[::-1], 3))
    outs = []
    for zc in (0, 5, 2 * n + 1, 61, 0):
        ctx = _ctx(grid, n, h, tau, bc, zchunk=zc)
        y = dev(np.zeros(grid[::-1]))
        ctx.apply(u, y)
        outs.append(host(y))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_rhs_matches_oracle(bc, dt):
    grid, n, tau = (67, 29, 31), 3, 3e-3
    u = rounded(normal_field(grid[::-1], 1), dt)
    q = rounded(normal_field(grid[::-1], 2), dt)
    ctx = _ctx(grid, n, (0.1, 0.1, 0.1), tau, bc)
    b = dev(np.zeros(grid[::-1]), dt)
    ctx.rhs(dev(u, dt), dev(q, dt), b)
    v = u + tau * q
    ref = op.rhs(u, q, n, tau, bc)
    scale = op.mass_apply(np.abs(u) + tau * np.abs(q), n, bc)
    tol = op_tolerance(n, dt, scale) + (np.abs(ref) * 2.0 ** -24 if dt == "f32" else 0)
    assert np.all(np.abs(host(b) - ref) <= tol)
    b0 = dev(np.zeros(grid[::-1]), dt)
    ctx.rhs(dev(u, dt), None, b0)  # q = NULL means f = 0
    ref0 = op.mass_apply(u, n, bc)
    assert np.all(np.abs(host(b0) - ref0) <= op_tolerance(n, dt, op.mass_apply(np.abs(u), n, bc)) +
                  (np.abs(ref0) * 2.0 ** -24 if dt == "f32" else 0))


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_residual_and_dot(bc):
    grid, n, h, tau = (45, 33, 19), 3, (0.05, 0.04, 0.06), 1e-2
    x = normal_field(grid[::-1], 4)
    b = normal_field(grid[::-1], 5)
    ctx = _ctx(grid, n, h, tau, bc)
    r = dev(np.zeros(grid[::-1]))
    rn, bn = ctx.residual(dev(x), dev(b), r)
    ref = b - op.apply(x, n, h, tau, bc)
    assert np.allclose(host(r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert abs(rn - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    assert abs(bn - np.linalg.norm(b)) <= 1e-13 * np.linalg.norm(b)
    r32 = dev(np.zeros(grid[::-1]), "f32")
    rn2, _ = ctx.residual(dev(x), dev(b), r32)
    assert rn2 == rn
    assert np.allclose(host(r32), ref, rtol=2 ** -23, atol=0)
    d1 = ctx.dot(dev(x), dev(b))
    assert abs(d1 - float(np.sum(x * b))) <= 1e-12 * np.sum(np.abs(x * b))
    assert ctx.dot(dev(x), dev(b)) == d1  # bitwise reproducible
    xf = rounded(x, "f32")
    assert abs(ctx.dot(dev(xf, "f32"), dev(xf, "f32")) - float(np.sum(xf * xf))) <= 1e-12 * np.sum(xf * xf)


def test_convert_rounds_to_nearest_even():
    from oracle.rounding import to_bf16
    grid = (41, 9, 10)
    ctx = _ctx(grid, 1, (1, 1, 1), 1.0, "periodic")
    x = normal_field(grid[::-1], 9) * 10.0 ** np.random.default_rng(1).integers(-20, 20, grid[::-1])
    xd = dev(x)
    xb = dev(np.zeros(grid[::-1]), "bf16")
    ctx.convert(xd, xb)
    # f64 -> bf16 goes through fp32 first
    assert np.array_equal(host(xb), to_bf16(x.astype(np.float32)))
    xf = dev(np.zeros(grid[::-1]), "f32")
    ctx.convert(xd, xf)
    assert np.array_equal(host(xf), x.astype(np.float32).astype(np.float64))


def test_apply_rejects_unsupported_and_missing_workspace():
    grid = (16, 16, 16)
    c = tbs.Context(grid, 3, (1, 1, 1), 1.0, "dirichlet")
    u = dev(np.zeros(grid[::-1]))
    y = dev(np.zeros(grid[::-1]), "bf16")
    with pytest.raises(tbs.TbsError):
        c.apply(u, y)
    with pytest.raises(tbs.TbsError):
        c.residual(u, u.clone())  # no workspace bound
