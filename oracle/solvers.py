"""Iterative solvers of the implicit step (oracle; test infrastructure only).

Paper, Sec. 2.5 (pipeline step 3): the discrete system F(c) = t is solved by the conjugate
gradient method; the leg experiment of Sec. 3 uses CG with a Jacobi preconditioner.  For the
constant-coefficient operator diag(A) is a constant times I, so Jacobi scaling leaves the CG
iterates unchanged and is omitted.

cg()      Hestenes-Stiefel CG; stops when ||b - A x|| (recursive residual) <= rtol ||b||.
refine()  mixed-precision iterative refinement (Moler 1967; CG form of Carson & Higham 2018):
          outer residual in FP64, inner correction solve by any solver to relative tolerance eta.
"""
import numpy as np


def cg(apply_fn, b, x0, rtol, max_iter, fixed_iters=None):
    """Plain CG.  If fixed_iters is given, exactly that many iterations run (no stopping test).

    Returns (x, iters, rel_res_history), rel_res = ||r_k|| / ||b|| with the recursive r_k.
    b = 0 gives x = 0 after zero iterations.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.sqrt(np.sum(b * b)))
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0]
    r = b - apply_fn(x)
    p = r.copy()
    rr = float(np.sum(r * r))
    hist = [np.sqrt(rr) / bnorm]
    k = 0
    limit = fixed_iters if fixed_iters is not None else max_iter
    while k < limit:
        if fixed_iters is None and np.sqrt(rr) <= rtol * bnorm:
            break
        q = apply_fn(p)
        pq = float(np.sum(p * q))
        if not np.isfinite(pq) or pq <= 0.0:
            raise FloatingPointError("CG breakdown: p^T A p <= 0 or not finite")
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.sum(r * r))
        beta = rr_new / rr
        rr = rr_new
        p = r + beta * p
        k += 1
        hist.append(np.sqrt(rr) / bnorm)
    return x, k, hist


def refine(apply_fn, b, x0, rtol, inner_solve, max_sweeps=10):
    """Iterative refinement: r = b - A x (FP64); stop if ||r|| <= rtol ||b||; s = ||r||;
    d = inner_solve(r / s); x += s d.  Returns (x, sweeps, final FP64 relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.sqrt(np.sum(b * b)))
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    sweeps = 0
    while True:
        r = b - apply_fn(x)
        rn = float(np.sqrt(np.sum(r * r)))
        if rn <= rtol * bnorm or sweeps >= max_sweeps:
            return x, sweeps, rn / bnorm
        d = inner_solve(r / rn)
        x = x + rn * d
        sweeps += 1


def rel_residual(apply_fn, b, x):
    """||b - A x||_2 / ||b||_2 in FP64 on coefficient vectors (0 for b = 0 and x = 0)."""
    b = np.asarray(b, dtype=np.float64)
    r = b - apply_fn(np.asarray(x, dtype=np.float64))
    bn = float(np.sqrt(np.sum(b * b)))
    rn = float(np.sqrt(np.sum(r * r)))
    return rn / bn if bn > 0 else rn
