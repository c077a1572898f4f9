"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds none of the method's arithmetic: it only draws random numbers and evaluates
analytic fields (Gaussians, sine modes) at node positions.  Mass-smoothing passes named in the
workload recipes are applied by the consumer (the oracle on the host, the library on the
device), never here.

Node positions (a reading of the unit-cube workloads): Dirichlet grids of N coefficients use
x_i = (i + 1) h with h = 1 / (N + 1) (zero-extended nodes sit at 0 and 1); periodic grids use
x_i = i h with h = 1 / N unless a spacing is given explicitly.  Arrays are [z, y, x].
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    grid: tuple            # (Nx, Ny, Nz)
    degree: int
    bc: str                # "periodic" | "dirichlet"
    h: tuple               # (hx, hy, hz)
    tau: float
    steps: int
    seed: int
    rtol: float
    smooth_passes: int = 0
    notes: str = ""
    degrees: tuple = field(default=())


def _h_dirichlet(N):
    return 1.0 / (N + 1)


HEAT_32_PERIODIC = Workload(
    "heat32_periodic_cubic", (32, 32, 32), 3, "periodic", (1 / 32,) * 3, 1e-3, 1, 1, 1e-10,
    smooth_passes=2, notes="N(0,1) + 2 mass passes + 4 sine modes, f = 0, FP64 CG to 1e-10")
HEAT_256_DIRICHLET = Workload(
    "heat256_dirichlet_cubic", (256, 256, 256), 3, "dirichlet", (1 / 257,) * 3, 1e-4, 10, 2, 1e-8,
    smooth_passes=3, notes="U[-1,1] + 3 mass passes, Gaussian source sigma 0.1 amplitude 10")
HEAT_928_DIRICHLET = Workload(
    "heat928_dirichlet_cubic", (928, 928, 928), 3, "dirichlet", (1 / 929,) * 3, 1e-5, 100, 3, 1e-8,
    notes="sum of 16 Gaussians, sigma in [0.02, 0.1], amplitudes N(0,1), f = 0")
HEAT_1024x512x256_PERIODIC = Workload(
    "heat1024x512x256_periodic", (1024, 512, 256), 3, "periodic", (1 / 512,) * 3, 5e-5, 20, 4, 1e-8,
    smooth_passes=2, notes="N(0,1) + 2 mass passes, f = 0", degrees=(2, 3, 5))
HEAT_128_TRAIN = Workload(
    "heat128_dirichlet_train", (128, 128, 128), 3, "dirichlet", (1 / 129,) * 3, 1e-4, 10, 5, 1e-10,
    notes="learned-guess training set: Gaussian-sum fields and 1-4 Gaussian sources")
HEAT_512_EVAL = Workload(
    "heat512_dirichlet_eval", (512, 512, 512), 3, "dirichlet", (1 / 513,) * 3, 1e-4, 50, 55, 1e-8,
    notes="learned vs plain initial guess, CG to 1e-8")

ALL = (HEAT_32_PERIODIC, HEAT_256_DIRICHLET, HEAT_928_DIRICHLET, HEAT_1024x512x256_PERIODIC,
       HEAT_128_TRAIN, HEAT_512_EVAL)


def node_coords(N, bc, h):
    i = np.arange(N, dtype=np.float64)
    return (i + 1.0) * h if bc == "dirichlet" else i * h


def normal_field(shape_zyx, seed):
    return np.random.default_rng(seed).standard_normal(shape_zyx)


def uniform_field(shape_zyx, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape_zyx)


def sine_modes(grid, h, seed, count=4, kmax=4):
    """sum of `count` modes sin(2 pi (mx x + my y + mz z)), m_d uniform in 1..kmax, amplitude 1."""
    rng = np.random.default_rng(seed)
    Nx, Ny, Nz = grid
    x = np.arange(Nx) * h[0]
    y = np.arange(Ny) * h[1]
    z = np.arange(Nz) * h[2]
    out = np.zeros((Nz, Ny, Nx))
    for _ in range(count):
        mx, my, mz = rng.integers(1, kmax + 1, size=3)
        out += np.sin(2 * np.pi * (mz * z[:, None, None] + my * y[None, :, None] + mx * x[None, None, :]))
    return out


def gaussian_params(seed, count, sigma_lo, sigma_hi, amp_scale, center_lo, center_hi, amp_normal=True):
    """Parameters (a, sigma, cx, cy, cz) of a Gaussian sum, one row per term."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(count) * amp_scale if amp_normal else np.full(count, float(amp_scale))
    s = rng.uniform(sigma_lo, sigma_hi, size=count)
    c = rng.uniform(center_lo, center_hi, size=(count, 3))
    return np.column_stack([a, s, c])


def gaussian_sum(grid, bc, h, params, xp=np, device=None, dtype=None):
    """sum_i a_i exp(-|x - c_i|^2 / (2 sigma_i^2)) at the node positions; separable per term.

    xp is numpy (host) or torch (device arrays; pass device and dtype)."""
    Nx, Ny, Nz = grid
    coords = [node_coords(N, bc, hd) for N, hd in zip(grid, h)]
    if xp is np:
        out = np.zeros((Nz, Ny, Nx))
        for a, s, cx, cy, cz in params:
            gx = np.exp(-(coords[0] - cx) ** 2 / (2 * s * s))
            gy = np.exp(-(coords[1] - cy) ** 2 / (2 * s * s))
            gz = np.exp(-(coords[2] - cz) ** 2 / (2 * s * s))
            out += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        return out
    import torch
    out = torch.zeros((Nz, Ny, Nx), device=device, dtype=dtype)
    for a, s, cx, cy, cz in params:
        gx = torch.from_numpy(a * np.exp(-(coords[0] - cx) ** 2 / (2 * s * s))).to(device=device, dtype=dtype)
        gy = torch.from_numpy(np.exp(-(coords[1] - cy) ** 2 / (2 * s * s))).to(device=device, dtype=dtype)
        gz = torch.from_numpy(np.exp(-(coords[2] - cz) ** 2 / (2 * s * s))).to(device=device, dtype=dtype)
        out.add_(gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    return out


def initial_field_gaussians(w, seed_offset=0):
    """16-term Gaussian sum of the 928^3 / learned-guess recipes (parameters only)."""
    return gaussian_params(w.seed * 1000 + seed_offset, 16, 0.02, 0.1, 1.0, 0.1, 0.9)


def source_gaussians(seed, count=None):
    """1-4 Gaussian sources, sigma in [0.05, 0.15], amplitudes 10 N(0,1)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 5)) if count is None else count
    return gaussian_params(seed + 7919, k, 0.05, 0.15, 10.0, 0.2, 0.8)


def source_256(seed):
    """One Gaussian source, sigma 0.1, amplitude 10, centre uniform in [0.2, 0.8]^3."""
    rng = np.random.default_rng(seed + 104729)
    c = rng.uniform(0.2, 0.8, size=3)
    return np.array([[10.0, 0.1, c[0], c[1], c[2]]])


def cnn_init(seed, layers=((2, 16), (16, 16), (16, 16), (16, 1)), last_scale=0.1):
    """He-normal initial weights (std sqrt(2 / fan_in)), zero biases, last layer scaled by 0.1.
    Flat fp32 vector in the order W1, b1, W2, b2, W3, b3, W4, b4."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(layers):
        std = np.sqrt(2.0 / (ci * 27))
        W = rng.standard_normal((co, ci, 3, 3, 3)) * std
        if li == len(layers) - 1:
            W *= last_scale
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)
