"""Pins of the learned-guess network oracle: torch's CPU conv3d and autograd, central finite
differences, the closed-form first Adam step and known bf16 roundings."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import cnn
from oracle.rounding import to_bf16
from workloads import cnn_init, normal_field


def _torch_conv(x, W, b, circular):
    xt = torch.from_numpy(x)[None]
    if circular:
        xt = F.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular")
        return F.conv3d(xt, torch.from_numpy(W), None if b is None else torch.from_numpy(b))[0].numpy()
    return F.conv3d(xt, torch.from_numpy(W), None if b is None else torch.from_numpy(b), padding=1)[0].numpy()


@pytest.mark.parametrize("circular", [False, True])
def test_conv_and_adjoints_match_torch(circular):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 6, 7))
    W = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.allclose(cnn.conv3d(x, W, b, circular), _torch_conv(x, W, b, circular), atol=1e-12)
    # adjoints through torch autograd
    g = rng.standard_normal((4, 5, 6, 7))
    xt = torch.from_numpy(x).requires_grad_(True)
    Wt = torch.from_numpy(W).requires_grad_(True)
    inp = xt[None]
    if circular:
        out = F.conv3d(F.pad(inp, (1, 1, 1, 1, 1, 1), mode="circular"), Wt)
    else:
        out = F.conv3d(inp, Wt, padding=1)
    (out[0] * torch.from_numpy(g)).sum().backward()
    assert np.allclose(cnn.conv3d_data_grad(g, W, circular), xt.grad.numpy(), atol=1e-11)
    dW, db = cnn.conv3d_weight_grad(x, g, circular)
    assert np.allclose(dW, Wt.grad.numpy(), atol=1e-11)
    assert np.allclose(db, g.sum(axis=(1, 2, 3)))


def test_param_count():
    assert cnn.N_PARAMS == 15169
    assert cnn_init(1).size == 15169


@pytest.mark.parametrize("circular", [False, True])
def test_gradient_matches_central_differences(circular):
    # unrounded network (plain FP64) on a 6^3 x 2-channel problem
    x0 = normal_field((2, 6, 6, 6), 3)
    theta = cnn_init(4).astype(np.float64)
    theta[-1] = 0.05
    theta[cnn.LAYERS[0][0] * 16 * 27: cnn.LAYERS[0][0] * 16 * 27 + 16] = 0.1  # nonzero b1
    target = normal_field((1, 6, 6, 6), 5)
    loss, g = cnn.loss_and_grad(x0, theta, target, circular, rounding=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(theta.size, 40, replace=False), [theta.size - 1, 880, 13900]])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (cnn.loss_only(x0, tp, target, circular, False) - cnn.loss_only(x0, tm, target, circular, False)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_rounded_forward_matches_torch_chain():
    # the rounded network equals torch conv3d + erf GELU applied on the same bf16 values
    x0 = normal_field((2, 5, 6, 4), 8)
    theta = cnn_init(9)
    params = [(to_bf16(W), b) for W, b in cnn.unpack(theta)]
    a = to_bf16(x0)
    for li, (W, b) in enumerate(params):
        z = _torch_conv(a, W, b, False)
        a = to_bf16(0.5 * z * (1 + torch.erf(torch.from_numpy(z) / np.sqrt(2)).numpy())) if li < 3 else z
    k1 = np.array([0.25, 0.5, 0.25])
    K = np.einsum("i,j,k->ijk", k1, k1, k1)[None, None]
    for _ in range(cnn.SMOOTH_PASSES):
        a = _torch_conv(a, K, None, False)
    assert np.allclose(cnn.forward(x0, theta, False), a, atol=1e-10)


@pytest.mark.parametrize("circular", [False, True])
def test_output_filter_symbol_and_adjoint(circular):
    # a Fourier mode on a periodic grid is scaled by prod_d cos^4(w_d / 2); the filter is symmetric
    N = 16
    x = np.arange(N)
    w = [2 * np.pi * k / N for k in (1, 3, 5)]
    mode = np.cos(w[2] * x[:, None, None] + w[1] * x[None, :, None] + w[0] * x[None, None, :])[None]
    if circular:
        expect = np.prod([np.cos(wi / 2) ** (2 * cnn.SMOOTH_PASSES) for wi in w])
        assert np.allclose(cnn.smooth(mode, True), expect * mode, atol=1e-13)
    a, b = normal_field((1, 7, 6, 5), 1), normal_field((1, 7, 6, 5), 2)
    assert abs(np.sum(cnn.smooth(a, circular) * b) - np.sum(a * cnn.smooth(b, circular))) < 1e-12


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    th, g = rng.standard_normal(50), rng.standard_normal(50)
    t1, m, v = cnn.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15)


@pytest.mark.parametrize("steps", [2, 3, 5])
def test_adam_constant_gradient_closed_form(steps):
    # with a constant gradient g from zero moments the bias-corrected moments are exactly
    # m_hat = g and v_hat = g^2 at every step t, so theta_t = theta_0 - t lr g / (|g| + eps):
    # a wrong bias-correction exponent for t > 1 changes m_hat / sqrt(v_hat) and fails this
    rng = np.random.default_rng(5)
    th0, g = rng.standard_normal(40), rng.standard_normal(40) * 10.0 ** rng.integers(-4, 2, 40)
    th, m, v = th0.copy(), np.zeros(40), np.zeros(40)
    for t in range(1, steps + 1):
        th, m, v = cnn.adam_step(th, g, m, v, t, lr=2e-3)
    assert np.allclose(th, th0 - steps * 2e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)


def test_bf16_rounding_known_values():
    ulp = 2.0 ** -7
    vals = np.array([1.0, 1 + ulp / 2, 1 + 1.5 * ulp, 1 + 0.75 * ulp, -3.0, 0.0, 1e-40])
    want = np.array([1.0, 1.0, 1 + 2 * ulp, 1 + ulp, -3.0, 0.0, None], dtype=object)
    got = to_bf16(vals)
    for g_, w_ in zip(got[:-1], want[:-1]):
        assert g_ == w_
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    rand = np.random.default_rng(3).standard_normal(10000) * 10.0 ** np.random.default_rng(4).integers(-30, 30, 10000)
    ref2 = torch.tensor(rand, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(to_bf16(rand), ref2)
