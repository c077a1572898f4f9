"""The network kernels' GELU: Phi(-y) = t 2^(P(t) - y^2 / (2 ln 2)), t = 1 / (1 + c y), with the
coefficients written in net.hip.  Checked on the host against scipy's normal log-CDF (relative error
of the tail below 1.3e-6) and, in fp32 arithmetic, against the exact GELU rounded to bf16."""
import os
import re

import numpy as np
import pytest

scipy_special = pytest.importorskip("scipy.special")

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1904_03057_amd", "csrc",
                   "net.hip")


def kernel_coefficients():
    text = open(SRC).read()
    body = text[text.index("__device__ __forceinline__ float gelu_f(float x)"):]
    body = body[:body.index("}\n")]
    c = float(re.search(r"rcpf\(fmaf\(([-+0-9.e]+)f", body).group(1))
    first = float(re.search(r"float p = ([-+0-9.e]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fmaf\(p, t, ([-+0-9.e]+)f\);", body)]
    scale = float(re.search(r"fmaf\(y \* y, ([-+0-9.e]+)f, p\)", body).group(1))
    return c, [first] + rest, scale


def test_tail_relative_error():
    c, P, scale = kernel_coefficients()
    assert len(P) == 7 and abs(scale + 0.5 / np.log(2)) < 1e-12
    y = np.linspace(0.0, 14.0, 200001)
    t = 1.0 / (1.0 + c * y)
    q = t * np.exp2(np.polyval(P, t) + scale * y * y)
    ref = np.exp(scipy_special.log_ndtr(-y))
    assert np.max(np.abs(q / ref - 1.0)) < 1.3e-6


def test_fp32_gelu_matches_exact_in_bf16():
    c, P, scale = kernel_coefficients()
    f = np.float32
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 200000), rng.normal(0, 3, 200000), np.linspace(-9, 9, 20001)]).astype(f)
    y = np.abs(x)
    t = (f(1) / (f(c) * y + f(1))).astype(f)
    p = f(P[0])
    for k in P[1:]:
        p = (p * t + f(k)).astype(f)
    q = (t * np.exp2((y * y * f(scale) + p).astype(f))).astype(f)
    g = (np.maximum(x, f(0)) - y * q).astype(f)
    xd = x.astype(np.float64)
    exact = 0.5 * xd * scipy_special.erfc(-xd / np.sqrt(2.0))

    def bf16(v):
        u = v.astype(np.float32).view(np.uint32).astype(np.uint64)
        return (u + 0x7FFF + ((u >> 16) & 1)) >> 16

    mism = np.mean(bf16(g) != bf16(exact))
    assert mism < 2e-3, mism
    rel = np.abs(g - exact) / np.maximum(np.abs(exact), 1e-30)
    assert np.max(rel[np.abs(exact) > 1e-30]) < 1e-4
