"""Helpers of the GPU tests: device transfer, rounding of inputs, and the tolerance of an
evaluation of A u in a given precision."""
import numpy as np

EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


def dev(a, dtype="f64"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    td = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    return t.to(td).to("cuda").contiguous()


def host(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def rounded(a, dtype):
    """The values a tensor of this dtype holds (what the oracle must be given)."""
    import torch
    td = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(td).to(torch.float64).numpy()


def op_tolerance(n, compute, scale):
    """Elementwise bound for any evaluation order of the 7-pass cascade in precision `compute`:
    gamma_K * (|A| |u|) with K = 4(2n + 4) operations along the longest chain (generous)."""
    k = 4 * (2 * n + 4)
    e = EPS[compute]
    return k * e / (1 - k * e) * scale
