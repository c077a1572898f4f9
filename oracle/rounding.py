"""bf16 rounding used at the documented rounding points (oracle; test infrastructure only).

bfloat16 keeps the top 16 bits of an IEEE binary32.  Round-to-nearest-even on the bit pattern:
add 0x7FFF plus the lowest kept bit, then truncate.  NaN is kept quiet.  Values are returned as
float64 that are exactly representable in bf16, so FP64 arithmetic on them is exact on input.
"""
import numpy as np


def to_bf16(x):
    a = np.asarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (rounded & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    out = np.where(nan, np.float32(np.nan), out)
    return out.astype(np.float64)


def to_f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)
