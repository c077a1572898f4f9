"""Fit of the normal tail used by the GELU epilogue of the network kernels.

Phi(-y) (y >= 0) is written as t * 2^(P(t) - y^2 / (2 ln 2)) with t = 1 / (1 + c y) and P a
polynomial of degree 6; P is fitted to log2(Phi(-y) / t) + y^2 / (2 ln 2) on y in [0, 14] by least
squares, reweighted iteratively toward the minimax solution, and its coefficients are rounded to
fp32.  Prints a C initialiser for the kernel source and the maximum relative error of Phi(-y)
(evaluated in FP64 with the rounded coefficients).

    python paper_1904_03057_amd/fit_gelu.py
"""
import numpy as np
from scipy.special import log_ndtr

DEG = 6
YMAX = 14.0
L2E = 1.0 / np.log(2.0)


def fit(c, iters=40):
    y = np.linspace(0.0, YMAX, 200001)
    t = 1.0 / (1.0 + c * y)
    f = log_ndtr(-y) * L2E - np.log2(t) + 0.5 * y * y * L2E
    V = np.vander(t, DEG + 1)
    w = np.ones_like(t)
    for _ in range(iters):
        coef, *_ = np.linalg.lstsq(V * w[:, None], f * w, rcond=None)
        e = V @ coef - f
        w = w * (1.0 + 5.0 * np.abs(e) / np.abs(e).max())
        w /= w.mean()
    return coef.astype(np.float32)


def rel_error(c, coef):
    y = np.linspace(0.0, YMAX, 400001)
    t = 1.0 / (1.0 + np.float64(np.float32(c)) * y)
    P = np.polyval(coef.astype(np.float64), t)
    q = t * np.exp2(P - 0.5 * y * y * L2E)
    ref = np.exp(log_ndtr(-y))
    return float(np.max(np.abs(q / ref - 1.0)))


def main():
    best = None
    for c in np.linspace(0.25, 0.31, 25):
        coef = fit(c)
        err = rel_error(c, coef)
        if best is None or err < best[0]:
            best = (err, float(np.float32(c)), coef)
    err, c, coef = best
    print("c = %.9ef" % c)
    print("P (highest degree first) = {" + ", ".join("%.9ef" % v for v in coef) + "}")
    print("max relative error of Phi(-y): %.3e" % err)


if __name__ == "__main__":
    main()
