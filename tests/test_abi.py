"""Host-side checks of the C ABI (no GPU): the library loads, exports every declared symbol, and
rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_1904_03057_amd as tbs

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tbs.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tbs_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    syms = declared_symbols()
    assert len(syms) >= 20
    lib = tbs.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(tbs.EXPORTS)


def _setup(grid=(16, 16, 16), n=3, h=(0.1, 0.1, 0.1), tau=1e-3, bc=tbs.DIRICHLET):
    p = ctypes.c_void_p()
    rc = tbs.lib().tbs_setup(ctypes.byref(p), (ctypes.c_int64 * 3)(*grid), n, (ctypes.c_double * 3)(*h), tau, bc, None)
    return rc, p


@pytest.mark.parametrize("kw", [dict(n=0), dict(n=6), dict(tau=0.0), dict(tau=-1.0), dict(h=(0.1, 0.0, 0.1)),
                                dict(grid=(6, 16, 16)), dict(bc=7), dict(grid=(16, 16, 2), n=1),
                                dict(tau=float("nan"))])
def test_setup_rejects_bad_arguments(kw):
    rc, p = _setup(**kw)
    assert rc == tbs.E_INVAL and not p


def test_valid_setup_and_workspace_sizes_without_gpu():
    rc, p = _setup(grid=(33, 17, 9), n=2)
    assert rc == tbs.OK
    lib = tbs.lib()
    base = lib.tbs_workspace_bytes(p, -1)
    N = 33 * 17 * 9
    assert base > 0
    assert lib.tbs_workspace_bytes(p, tbs.PREC_FP64) >= base + 7 * N * 8
    assert lib.tbs_workspace_bytes(p, tbs.PREC_MIXED) >= base + N * 8 + 5 * N * 4
    assert lib.tbs_workspace_bytes(p, 9) == 0
    m = (ctypes.c_double * 3)()
    s = (ctypes.c_double * 3)()
    assert lib.tbs_taps(p, m, s) == tbs.OK
    # the library's own FP64 taps equal the exact rationals (n = 2: 11/20, 13/60, 1/120 ; 1, -1/3, -1/6)
    assert list(m) == pytest.approx([11 / 20, 13 / 60, 1 / 120], abs=1e-15)
    assert list(s) == pytest.approx([1.0, -1 / 3, -1 / 6], abs=1e-15)
    lib.tbs_destroy(p)


def test_calls_validate_pointers_before_hip():
    rc, p = _setup()
    lib = tbs.lib()
    aligned = ctypes.c_void_p(1 << 20)      # never dereferenced: validation fails first
    misaligned = ctypes.c_void_p((1 << 20) + 8)
    assert lib.tbs_apply(p, None, tbs.F64, aligned, tbs.F64) == tbs.E_INVAL
    assert lib.tbs_apply(p, misaligned, tbs.F64, aligned, tbs.F64) == tbs.E_INVAL
    assert lib.tbs_apply(p, aligned, tbs.F64, aligned, tbs.F64) == tbs.E_INVAL          # aliasing
    assert lib.tbs_apply(p, aligned, tbs.F64, ctypes.c_void_p(1 << 21), tbs.BF16) == tbs.E_INVAL  # bad dtype pair
    assert lib.tbs_rhs(p, aligned, None, ctypes.c_void_p(1 << 21), tbs.BF16) == tbs.E_INVAL
    assert lib.tbs_cg_step(p, 3, None, None) == tbs.E_STATE
    assert lib.tbs_timestep(p, aligned, None, ctypes.c_void_p(1 << 21), 9, 1e-8, 10, None, None) == tbs.E_INVAL
    # valid pointers but no workspace bound -> NOMEM before any HIP call
    assert lib.tbs_timestep(p, aligned, None, ctypes.c_void_p(1 << 21), tbs.PREC_FP64, 1e-8, 10, None, None) == tbs.E_NOMEM
    assert lib.tbs_bind_workspace(p, misaligned, 1 << 30) == tbs.E_INVAL
    assert lib.tbs_bind_workspace(p, aligned, 16) == tbs.E_NOMEM
    assert lib.tbs_strerror(tbs.E_BREAKDOWN).startswith(b"CG breakdown")
    lib.tbs_destroy(p)


def test_transform_setup_validation_without_gpu():
    lib = tbs.lib()
    p = ctypes.c_void_p()
    g = (ctypes.c_int64 * 3)(16, 16, 16)
    for deg in (0, 1, 6):
        assert lib.tbs_transform_setup(ctypes.byref(p), g, deg, tbs.DIRICHLET, None) == tbs.E_INVAL and not p
    small = (ctypes.c_int64 * 3)(16, 4, 16)  # degree 5: half-width 2 needs N_d >= 5
    assert lib.tbs_transform_setup(ctypes.byref(p), small, 5, tbs.PERIODIC, None) == tbs.E_INVAL and not p
    assert lib.tbs_transform_setup(ctypes.byref(p), g, 3, tbs.DIRICHLET, None) == tbs.OK and p
    aligned = ctypes.c_void_p(1 << 20)
    # a transform context refuses the time step, and the transform calls refuse a solver context
    assert lib.tbs_timestep(p, aligned, None, ctypes.c_void_p(1 << 21), tbs.PREC_FP64, 1e-8, 10, None,
                            None) == tbs.E_STATE
    rc, s = _setup()
    assert rc == tbs.OK
    assert lib.tbs_transform_eval(s, aligned, ctypes.c_void_p(1 << 21), tbs.F64) == tbs.E_STATE
    lib.tbs_destroy(s)
    lib.tbs_destroy(p)


def test_set_opts_validation_without_gpu():
    rc, p = _setup()
    lib = tbs.lib()
    good = tbs.Opts(1e-6, 500, 12, 4, 0, 0, 0, 1, 0, 1e-2, 1)
    assert lib.tbs_set_opts(p, ctypes.byref(good)) == tbs.OK
    assert lib.tbs_set_opts(p, None) == tbs.OK
    for field, bad in (("guess_backoff", 3), ("guess_backoff", -1), ("fused_cg", 2), ("inner_rtol", 0.0),
                       ("coarse_rtol", 1.0), ("poll_every", -1), ("guess_test", 2), ("guess_test", -1), ("fused_rhs", 2)):
        o = tbs.Opts(1e-6, 500, 12, 4, 0, 0, 0, 1, 0, 1e-2, 0)
        setattr(o, field, bad)
        assert lib.tbs_set_opts(p, ctypes.byref(o)) == tbs.E_INVAL, field
    lib.tbs_destroy(p)


def test_residual_noalloc_validates_before_any_hip_call():
    lib = tbs.lib()
    a, b, r, nrm = (ctypes.c_void_p(256 * k) for k in (1, 2, 3, 4))
    rc, p = _setup(grid=(64, 64, 16), n=2)
    assert rc == tbs.OK
    lib.tbs_residual_noalloc.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int, ctypes.c_void_p]
    assert lib.tbs_residual_noalloc(p, a, b, r, tbs.F64, None) == tbs.E_INVAL          # no norms buffer
    assert lib.tbs_residual_noalloc(p, a, b, r, tbs.F64, ctypes.c_void_p(260)) == tbs.E_INVAL  # misaligned
    assert lib.tbs_residual_noalloc(p, a, b, a, tbs.F64, nrm) == tbs.E_INVAL            # r aliases x
    assert lib.tbs_residual_noalloc(p, a, b, r, tbs.BF16, nrm) == tbs.E_INVAL           # bad r dtype
    lib.tbs_destroy(p)
    # a plane of 19200 x 4800 points needs 300 * 300 residual workgroups (64 x 16 tiles): more than
    # the static buffer holds
    rc, p = _setup(grid=(64 * 300, 16 * 300, 16), n=2)
    assert rc == tbs.OK
    assert lib.tbs_residual_noalloc(p, a, b, r, tbs.F64, nrm) == tbs.E_INVAL
    assert b"static buffer" in tbs.lib().tbs_last_error()
    lib.tbs_destroy(p)


def test_setup_robin_validates_without_gpu():
    lib = tbs.lib()
    p = ctypes.c_void_p()
    g = lambda *a: (ctypes.c_int64 * 3)(*a)
    hh = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    # degree 3: every N_d >= 4 floor(n/2) + 2 + n = 9
    assert lib.tbs_setup_robin(ctypes.byref(p), g(9, 9, 9), 3, hh, 1e-3, 0.01, None) == tbs.OK and p
    lib.tbs_destroy(p)
    for args in ((g(8, 9, 9), 3, 0.01), (g(13, 14, 14), 4, 0.01), (g(16, 16, 16), 3, 0.0), (g(16, 16, 16), 3, -1.0),
                 (g(16, 16, 16), 6, 0.01), (g(16, 16, 16), 3, float("inf"))):
        p = ctypes.c_void_p()
        assert lib.tbs_setup_robin(ctypes.byref(p), args[0], args[1], hh, 1e-3, args[2], None) == tbs.E_INVAL
        assert not p
    # tbs_setup itself does not take the Robin boundary (it needs gamma)
    rc, p = _setup(bc=tbs.ROBIN)
    assert rc == tbs.E_INVAL
    # the coarse-grid guess is refused on a Robin box
    p = ctypes.c_void_p()
    assert lib.tbs_setup_robin(ctypes.byref(p), g(16, 16, 16), 3, hh, 1e-3, 0.01, None) == tbs.OK
    o = tbs.Opts(1e-6, 500, 12, 4, 0, 0, 0, 1, 1, 1e-2, 0, 0)
    assert lib.tbs_set_opts(p, ctypes.byref(o)) == tbs.E_INVAL
    lib.tbs_destroy(p)
