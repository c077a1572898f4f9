"""FP64 reference of the learned initial-guess network (oracle; test infrastructure only).

Not in the paper: the paper warm-starts CG from a coarse-grid solution (Sec. 3, leg example);
here a small 3-D CNN predicts the CG initial guess u^{k+1} - u^k from (u^k, f).

Network (4 layers, 3x3x3 cross-correlation, "same" padding: zero for Dirichlet grids, circular
for periodic grids):
    y1 = GELU(W1 * x0 + b1)   2 -> 16
    y2 = GELU(W2 * y1 + b2)  16 -> 16
    y3 = GELU(W3 * y2 + b3)  16 -> 16
    o  =      W4 * y3 + b4   16 -> 1
GELU is the exact erf form x/2 (1 + erf(x / sqrt 2)).  Parameter count 15,169.
The network output is followed by a fixed low-pass filter B^2, B = Bx By Bz with the binomial
taps [1/4, 1/2, 1/4] on each axis (zero padding / circular): a guess with grid-scale noise has
error in the modes where A's eigenvalues are smallest, which CG converges on slowly.  B is
symmetric, so the output gradient passes through the same filter.

Rounding points (matching the device kernels, which multiply bf16 x bf16 and accumulate in
fp32): every tensor that enters a product is rounded to bf16 first -- the inputs x0, the
weights, the stored activations y1..y3, and in the backward pass the output gradient and the
pre-activation gradients dz1..dz3.  Biases are only added, so they stay fp32.  Arithmetic here
is FP64 on those values.

Tensors are [C, Z, Y, X]; weights [C_out, C_in, 3, 3, 3] indexed (dz, dy, dx).
"""
import numpy as np
from scipy.special import erf

from .rounding import to_bf16

LAYERS = ((2, 16), (16, 16), (16, 16), (16, 1))
SMOOTH_PASSES = 2
N_PARAMS = sum(ci * co * 27 + co for ci, co in LAYERS)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def _shift(x, dz, dy, dx, circular):
    """s[c, z, y, x] = x[c, z+dz, y+dy, x+dx] with zero or circular padding."""
    if circular:
        return np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))
    C, Z, Y, X = x.shape
    out = np.zeros_like(x)

    def rng(d, N):
        return (slice(max(0, -d), N - max(0, d)), slice(max(0, d), N - max(0, -d)))

    (oz, iz), (oy, iy), (ox, ix) = rng(dz, Z), rng(dy, Y), rng(dx, X)
    out[:, oz, oy, ox] = x[:, iz, iy, ix]
    return out


def conv3d(x, W, b, circular):
    """out[co, p] = b[co] + sum_{ci, d} W[co, ci, d] x[ci, p + d - 1]."""
    Co = W.shape[0]
    out = np.zeros((Co,) + x.shape[1:], dtype=np.float64)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xs = _shift(x, kz - 1, ky - 1, kx - 1, circular)
                out += np.einsum("oc,czyx->ozyx", W[:, :, kz, ky, kx], xs)
    if b is not None:
        out += np.asarray(b, dtype=np.float64)[:, None, None, None]
    return out


def conv3d_data_grad(g, W, circular):
    """dx[ci, p] = sum_{co, d} W[co, ci, d] g[co, p - (d - 1)] (adjoint of conv3d in x)."""
    Ci = W.shape[1]
    out = np.zeros((Ci,) + g.shape[1:], dtype=np.float64)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                gs = _shift(g, 1 - kz, 1 - ky, 1 - kx, circular)
                out += np.einsum("oc,ozyx->czyx", W[:, :, kz, ky, kx], gs)
    return out


def conv3d_weight_grad(x, g, circular):
    """dW[co, ci, d] = sum_p g[co, p] x[ci, p + d - 1];  db[co] = sum_p g[co, p]."""
    Co, Ci = g.shape[0], x.shape[0]
    dW = np.zeros((Co, Ci, 3, 3, 3), dtype=np.float64)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xs = _shift(x, kz - 1, ky - 1, kx - 1, circular)
                dW[:, :, kz, ky, kx] = np.einsum("ozyx,czyx->oc", g, xs)
    return dW, g.sum(axis=(1, 2, 3))


def smooth(o, circular, passes=SMOOTH_PASSES):
    """B^passes o for o = [C, Z, Y, X]: binomial [1/4, 1/2, 1/4] along x, y and z."""
    o = np.asarray(o, dtype=np.float64)
    for _ in range(passes):
        for ax in (3, 2, 1):
            shape = [0, 0, 0]
            d = [0, 0, 0]
            d[ax - 1] = 1
            lo = _shift(o, -d[0], -d[1], -d[2], circular)
            hi = _shift(o, d[0], d[1], d[2], circular)
            o = 0.25 * lo + 0.5 * o + 0.25 * hi
    return o


def unpack(theta):
    """Flat parameter vector -> [(W1, b1), ..., (W4, b4)] (order: W then b per layer)."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = np.asarray(theta[o:o + co * ci * 27], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        o += co * ci * 27
        b = np.asarray(theta[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def forward(x0, theta, circular, keep=False, rounding=True):
    """x0 [2, Z, Y, X] -> o [1, Z, Y, X]; weights and x0 rounded to bf16, activations stored bf16.
    rounding=False runs the same network in plain FP64 (for finite-difference checks)."""
    rnd = to_bf16 if rounding else _identity
    params = [(rnd(W), b) for W, b in unpack(np.asarray(theta, dtype=np.float32 if rounding else np.float64))]
    a = rnd(x0)
    acts, pre = [a], []
    for li, (W, b) in enumerate(params):
        z = conv3d(a, W, None, circular) + b[:, None, None, None]
        if li < 3:
            pre.append(z)
            a = rnd(gelu(z))
            acts.append(a)
        else:
            o = smooth(z, circular)
    if keep:
        return o, acts, pre
    return o


def loss_and_grad(x0, theta, target, circular, rounding=True):
    """MSE loss mean((o - t)^2) and its gradient w.r.t. the fp32 master weights theta.

    Backward rounding points: the output gradient and each dz are rounded to bf16 before the
    weight-gradient and data-gradient products, as on the device.  Bias gradients use the
    same rounded values.
    """
    rnd = to_bf16 if rounding else _identity
    params = [(rnd(W), b) for W, b in unpack(np.asarray(theta, dtype=np.float32 if rounding else np.float64))]
    o, acts, pre = forward(x0, theta, circular, keep=True, rounding=rounding)
    diff = o - target
    loss = float(np.mean(diff * diff))
    g = rnd(smooth(2.0 * diff / diff.size, circular))
    grads = [None] * 4
    for li in range(3, -1, -1):
        W, _ = params[li]
        dW, db = conv3d_weight_grad(acts[li], g, circular)
        grads[li] = (dW, db)
        if li > 0:
            dy = conv3d_data_grad(g, W, circular)
            g = rnd(dy * gelu_grad(pre[li - 1]))
    return loss, pack(grads)


def loss_only(x0, theta, target, circular, rounding=True):
    o = forward(x0, theta, circular, rounding=rounding)
    d = o - target
    return float(np.mean(d * d))


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), t = 1-based step count.  Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
