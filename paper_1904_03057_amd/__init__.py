"""Python binding of libtbs.so (MI355X tensor B-spline implicit heat step).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
PyTorch provides device memory and streams.  If the shared library has not been built the
import fails loudly; there is no fallback path.
"""
import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtbs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libtbs.so is not built: run `python paper_1904_03057_amd/build.py` "
                      "(or __graft_entry__.build()) first")

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Loading torch first
# makes the library bind to that already-loaded runtime, so one process never holds two HIP/HSA
# runtimes (the second one would not see the device).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_HIP, E_BREAKDOWN, E_STATE, W_NOT_CONVERGED = 0, -1, -2, -3, -4, -5, 1
PERIODIC, DIRICHLET, ROBIN = 0, 1, 2
F64, F32, BF16 = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_MIXED, PREC_MIXED_BF16 = 0, 1, 2, 3
NET_PARAMS = 15169

EXPORTS = [
    "tbs_setup", "tbs_destroy", "tbs_workspace_bytes", "tbs_bind_workspace", "tbs_taps", "tbs_set_opts",
    "tbs_apply", "tbs_rhs", "tbs_residual", "tbs_dot", "tbs_convert", "tbs_cg_begin", "tbs_cg_step",
    "tbs_timestep", "tbs_net_create", "tbs_net_destroy", "tbs_net_workspace_bytes", "tbs_net_bind_workspace",
    "tbs_net_set_weights", "tbs_net_get_weights", "tbs_net_set_hparams", "tbs_net_forward",
    "tbs_net_train_step", "tbs_net_conv_layer", "tbs_net_get_grad", "tbs_prof_enable", "tbs_prof_read", "tbs_strerror",
    "tbs_last_error", "tbs_transform_setup", "tbs_transform_eval", "tbs_transform_interp", "tbs_residual_noalloc",
    "tbs_setup_robin", "tbs_apply_varcoef", "tbs_stream_copy",
]
PROF_KINDS = ["apply_f64", "apply_f32", "apply_bf16_f32", "rhs_f64", "rhs_f32", "cg_fused_f64", "cg_fused_f32",
              "cg_fused_f32_bf16p", "residual_f64", "cg_update_f64", "cg_update_f32", "cg_iter_f32",
              "cg_iter_f32_bf16p", "varcoef_f64", "varcoef_f32", "cg_iter_f64", "rhs_resid_f64"]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("sweeps", ctypes.c_int), ("used_learned_guess", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res_fp64", ctypes.c_double), ("rel_res0", ctypes.c_double),
                ("rel_res_plain", ctypes.c_double), ("rel_res_learned", ctypes.c_double),
                ("used_coarse_guess", ctypes.c_int), ("coarse_iters", ctypes.c_int),
                ("rel_res_coarse", ctypes.c_double), ("skipped_learned_guess", ctypes.c_int),
                ("learned_gamma", ctypes.c_double), ("learned_saved_iters", ctypes.c_double),
                ("learned_cost_iters", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(ctypes.Structure):
    _fields_ = [("inner_rtol", ctypes.c_double), ("inner_max_iter", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("poll_every", ctypes.c_int), ("zchunk", ctypes.c_int),
                ("tile_order", ctypes.c_int), ("nt_store", ctypes.c_int), ("fused_cg", ctypes.c_int),
                ("coarse_guess", ctypes.c_int), ("coarse_rtol", ctypes.c_double), ("guess_backoff", ctypes.c_int),
                ("guess_test", ctypes.c_int), ("fused_rhs", ctypes.c_int)]


_vp, _i64p, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
_lib.tbs_setup.argtypes = [ctypes.POINTER(_vp), _i64p, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _vp]
_lib.tbs_setup_robin.argtypes = [ctypes.POINTER(_vp), _i64p, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double,
                                 _vp]
_lib.tbs_destroy.argtypes = [_vp]
_lib.tbs_destroy.restype = None
_lib.tbs_workspace_bytes.argtypes = [_vp, ctypes.c_int]
_lib.tbs_workspace_bytes.restype = ctypes.c_size_t
_lib.tbs_bind_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.tbs_taps.argtypes = [_vp, _dp, _dp]
_lib.tbs_set_opts.argtypes = [_vp, ctypes.POINTER(Opts)]
_lib.tbs_apply.argtypes = [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int]
_lib.tbs_rhs.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int]
_lib.tbs_apply_varcoef.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int]
_lib.tbs_transform_setup.argtypes = [ctypes.POINTER(_vp), _i64p, ctypes.c_int, ctypes.c_int, _vp]
_lib.tbs_transform_eval.argtypes = [_vp, _vp, _vp, ctypes.c_int]
_lib.tbs_transform_interp.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      _dp]
_lib.tbs_residual.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _dp, _dp]
_lib.tbs_residual_noalloc.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]
_lib.tbs_dot.argtypes = [_vp, _vp, _vp, ctypes.c_int, _dp]
_lib.tbs_convert.argtypes = [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int]
_lib.tbs_stream_copy.argtypes = [_vp, _vp, _vp, ctypes.c_size_t]
_lib.tbs_cg_begin.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double]
_lib.tbs_cg_step.argtypes = [_vp, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int)]
_lib.tbs_timestep.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _vp,
                              ctypes.POINTER(Stats)]
_lib.tbs_net_create.argtypes = [ctypes.POINTER(_vp), _vp]
_lib.tbs_net_destroy.argtypes = [_vp]
_lib.tbs_net_destroy.restype = None
_lib.tbs_net_workspace_bytes.argtypes = [_i64p, ctypes.c_int, ctypes.c_int]
_lib.tbs_net_workspace_bytes.restype = ctypes.c_size_t
_lib.tbs_net_bind_workspace.argtypes = [_vp, _i64p, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t]
_lib.tbs_net_set_weights.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]
_lib.tbs_net_get_weights.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]
_lib.tbs_net_set_hparams.argtypes = [_vp, ctypes.c_double, ctypes.c_double]
_lib.tbs_net_forward.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_double]
_lib.tbs_net_train_step.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_float)]
_lib.tbs_net_conv_layer.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp]
_lib.tbs_net_get_grad.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]
_lib.tbs_prof_enable.argtypes = [_vp, ctypes.c_int]
_lib.tbs_prof_read.argtypes = [_vp, ctypes.c_int, _dp, _dp, ctypes.POINTER(ctypes.c_int64)]
_lib.tbs_strerror.argtypes = [ctypes.c_int]
_lib.tbs_strerror.restype = ctypes.c_char_p
_lib.tbs_last_error.argtypes = []
_lib.tbs_last_error.restype = ctypes.c_char_p


class TbsError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = "%s: %s (%d): %s" % (where, _lib.tbs_strerror(code).decode(), code,
                                   (_lib.tbs_last_error() or b"").decode())
        super().__init__(msg)


def _check(rc, where, allow=(OK,)):
    if rc not in allow:
        raise TbsError(rc, where)
    return rc


def lib():
    return _lib


def _dtype_code(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


class Context:
    """One grid / degree / spacing / time step / boundary condition, bound to one HIP stream."""

    def __init__(self, grid, degree, h, tau, bc, stream=None, _no_stream=False):
        self._h = ctypes.c_void_p()
        if _no_stream:
            sh, self.stream = ctypes.c_void_p(None), None
        else:
            sh, self.stream = _stream_handle(stream)
        g = (ctypes.c_int64 * 3)(*grid)
        hh = (ctypes.c_double * 3)(*h)
        bcc = {"periodic": PERIODIC, "dirichlet": DIRICHLET}.get(bc, bc)
        _check(_lib.tbs_setup(ctypes.byref(self._h), g, degree, hh, tau, bcc, sh), "tbs_setup")
        self.grid, self.degree, self.h, self.tau, self.bc = tuple(grid), degree, tuple(h), tau, bcc
        self.shape = (grid[2], grid[1], grid[0])
        self._ws = None

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None) is not None and self._h:
            _lib.tbs_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, prec=-1):
        return int(_lib.tbs_workspace_bytes(self._h, prec))

    def bind_workspace(self, buf):
        _check(_lib.tbs_bind_workspace(self._h, _ptr(buf), buf.numel() * buf.element_size()), "tbs_bind_workspace")
        self._ws = buf

    def ensure_workspace(self, prec=-1):
        import torch
        need = self.workspace_bytes(prec)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            buf = torch.empty(need, dtype=torch.uint8, device="cuda")
            self.bind_workspace(buf)
        return self._ws

    def taps(self):
        m = (ctypes.c_double * (self.degree + 1))()
        s = (ctypes.c_double * (self.degree + 1))()
        _check(_lib.tbs_taps(self._h, m, s), "tbs_taps")
        return list(m), list(s)

    def set_opts(self, inner_rtol=1e-6, inner_max_iter=500, max_sweeps=12, poll_every=4, zchunk=0,
                 tile_order=0, nt_store=0, fused_cg=1, coarse_guess=0, coarse_rtol=1e-2, guess_backoff=0,
                 guess_test=0, fused_rhs=1):
        o = Opts(inner_rtol, inner_max_iter, max_sweeps, poll_every, zchunk, tile_order, nt_store, fused_cg,
                 coarse_guess, coarse_rtol, guess_backoff, guess_test, fused_rhs)
        _check(_lib.tbs_set_opts(self._h, ctypes.byref(o)), "tbs_set_opts")
        # options can change the workspace layout (partial-sum count, coarse-guess region): the
        # library drops its binding then; rebind the buffer if it still holds the minimum
        if self._ws is not None:
            buf, self._ws = self._ws, None
            if buf.numel() >= self.workspace_bytes(-1):
                self.bind_workspace(buf)

    def apply(self, u, y):
        _check(_lib.tbs_apply(self._h, _ptr(u), _dtype_code(u), _ptr(y), _dtype_code(y)), "tbs_apply")

    def apply_varcoef(self, u, d, m, y):
        """y = F(u) with the coefficient fields d (diffusion) and m (absorption) in the same basis."""
        _check(_lib.tbs_apply_varcoef(self._h, _ptr(u), _ptr(d), _ptr(m), _ptr(y), _dtype_code(y)),
               "tbs_apply_varcoef")

    def rhs(self, u_prev, q, b):
        _check(_lib.tbs_rhs(self._h, _ptr(u_prev), _ptr(q), _ptr(b), _dtype_code(b)), "tbs_rhs")

    def residual(self, x, b, r=None):
        rn, bn = ctypes.c_double(), ctypes.c_double()
        _check(_lib.tbs_residual(self._h, _ptr(x), _ptr(b), _ptr(r), F64 if r is None else _dtype_code(r),
                                 ctypes.byref(rn), ctypes.byref(bn)), "tbs_residual")
        return rn.value, bn.value

    def residual_noalloc(self, x, b, r=None, norms=None):
        """Allocation-free residual: writes ||b - A x||, ||b|| into the device tensor `norms`
        (2 float64 values; allocated here if None) without synchronising; returns `norms`."""
        import torch
        if norms is None:
            norms = torch.empty(2, dtype=torch.float64, device=x.device)
        _check(_lib.tbs_residual_noalloc(self._h, _ptr(x), _ptr(b), _ptr(r), F64 if r is None else _dtype_code(r),
                                         _ptr(norms)), "tbs_residual_noalloc")
        return norms

    def dot(self, a, b):
        out = ctypes.c_double()
        _check(_lib.tbs_dot(self._h, _ptr(a), _ptr(b), _dtype_code(a), ctypes.byref(out)), "tbs_dot")
        return out.value

    def convert(self, src, dst):
        _check(_lib.tbs_convert(self._h, _ptr(src), _dtype_code(src), _ptr(dst), _dtype_code(dst)), "tbs_convert")

    def stream_copy(self, src, dst):
        """dst <- src (same byte size) with the library's 16-byte streaming copy kernel."""
        nb = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nb:
            raise ValueError("src and dst sizes differ")
        _check(_lib.tbs_stream_copy(self._h, _ptr(src), _ptr(dst), nb), "tbs_stream_copy")

    def cg_begin(self, b, x, rtol):
        _check(_lib.tbs_cg_begin(self._h, _ptr(b), _ptr(x), _dtype_code(x), rtol), "tbs_cg_begin")

    def cg_step(self, n_iters, sync=True):
        """n_iters CG iterations; (relative recursive residual, completed iterations), or None
        without sync (no host read: with poll_every=0 the call is graph-capturable)."""
        if not sync:
            _check(_lib.tbs_cg_step(self._h, n_iters, None, None), "tbs_cg_step")
            return None
        rel, it = ctypes.c_double(), ctypes.c_int()
        _check(_lib.tbs_cg_step(self._h, n_iters, ctypes.byref(rel), ctypes.byref(it)), "tbs_cg_step")
        return rel.value, it.value

    def prof_enable(self, on=True):
        _check(_lib.tbs_prof_enable(self._h, int(on)), "tbs_prof_enable")

    def prof_read(self):
        """{kind: (total_ms, total_bytes, launches)} for every kind with launches."""
        out = {}
        for i, name in enumerate(PROF_KINDS):
            ms, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
            _check(_lib.tbs_prof_read(self._h, i, ctypes.byref(ms), ctypes.byref(by), ctypes.byref(n)), "tbs_prof_read")
            if n.value:
                out[name] = (ms.value, by.value, n.value)
        return out

    def timestep(self, u_prev, q, u_next, prec=PREC_FP64, rtol=1e-10, max_iter=1000, net=None):
        st = Stats()
        rc = _lib.tbs_timestep(self._h, _ptr(u_prev), _ptr(q), _ptr(u_next), prec, rtol, max_iter,
                               None if net is None else net.handle, ctypes.byref(st))
        _check(rc, "tbs_timestep", allow=(OK, W_NOT_CONVERGED))
        d = st.as_dict()
        d["converged"] = rc == OK
        return d


class RobinContext(Context):
    """Box domain with the Robin / penalty boundary branch (parameter gamma), N_d = Nc_d + 1 + 2 floor(n/2)
    coefficients per axis; apply, rhs, residual, CG and time steps as on a Context."""

    def __init__(self, grid, degree, h, tau, gamma, stream=None):
        self._h = ctypes.c_void_p()
        sh, self.stream = _stream_handle(stream)
        g = (ctypes.c_int64 * 3)(*grid)
        hh = (ctypes.c_double * 3)(*h)
        _check(_lib.tbs_setup_robin(ctypes.byref(self._h), g, degree, hh, tau, gamma, sh), "tbs_setup_robin")
        self.grid, self.degree, self.h, self.tau, self.bc, self.gamma = tuple(grid), degree, tuple(h), tau, ROBIN, gamma
        self.shape = (grid[2], grid[1], grid[0])
        self._ws = None


class Transform(Context):
    """Direct / indirect B-spline transforms of one grid, spline degree 2..5 and boundary condition."""

    def __init__(self, grid, degree, bc, stream=None):
        self._h = ctypes.c_void_p()
        sh, self.stream = _stream_handle(stream)
        g = (ctypes.c_int64 * 3)(*grid)
        bcc = {"periodic": PERIODIC, "dirichlet": DIRICHLET}.get(bc, bc)
        _check(_lib.tbs_transform_setup(ctypes.byref(self._h), g, degree, bcc, sh), "tbs_transform_setup")
        self.grid, self.degree, self.h, self.tau, self.bc = tuple(grid), degree, (1.0, 1.0, 1.0), 0.0, bcc
        self.shape = (grid[2], grid[1], grid[0])
        self._ws = None

    def eval(self, coef, samples):
        """samples = E coef (indirect transform); FP64 or FP32 arrays of the grid's shape."""
        _check(_lib.tbs_transform_eval(self._h, _ptr(coef), _ptr(samples), _dtype_code(samples)),
               "tbs_transform_eval")

    def interp(self, samples, coef, rtol=1e-13, max_iter=1000):
        """Direct transform: solve E coef = samples (FP64) starting from coef; returns (iters, rel_res)."""
        self.ensure_workspace(PREC_FP64)
        it, rel = ctypes.c_int(), ctypes.c_double()
        rc = _lib.tbs_transform_interp(self._h, _ptr(samples), _ptr(coef), rtol, max_iter, ctypes.byref(it),
                                       ctypes.byref(rel))
        _check(rc, "tbs_transform_interp", allow=(OK, W_NOT_CONVERGED))
        return it.value, rel.value


class Net:
    """Learned initial guess (3-D CNN, bf16 matrix-core kernels)."""

    def __init__(self, stream=None):
        self._h = ctypes.c_void_p()
        sh, self.stream = _stream_handle(stream)
        _check(_lib.tbs_net_create(ctypes.byref(self._h), sh), "tbs_net_create")
        self._ws = None
        self._ws_key = None

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None) is not None and self._h:
            _lib.tbs_net_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @staticmethod
    def workspace_bytes(grid, batch=1, training=False):
        g = (ctypes.c_int64 * 3)(*grid)
        return int(_lib.tbs_net_workspace_bytes(g, batch, int(training)))

    def ensure_workspace(self, grid, batch=1, training=False):
        import torch
        key = (tuple(grid), batch, bool(training))
        if self._ws_key == key:
            return
        need = self.workspace_bytes(grid, batch, training)
        self._ws = None
        buf = torch.empty(need, dtype=torch.uint8, device="cuda")
        g = (ctypes.c_int64 * 3)(*grid)
        _check(_lib.tbs_net_bind_workspace(self._h, g, batch, int(training), _ptr(buf), need), "tbs_net_bind_workspace")
        self._ws, self._ws_key = buf, key

    def set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(_lib.tbs_net_set_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size),
               "tbs_net_set_weights")

    def get_weights(self):
        import numpy as np
        w = np.zeros(NET_PARAMS, dtype=np.float32)
        _check(_lib.tbs_net_get_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size),
               "tbs_net_get_weights")
        return w

    def set_hparams(self, out_scale=1.0, lr=1e-3):
        _check(_lib.tbs_net_set_hparams(self._h, out_scale, lr), "tbs_net_set_hparams")

    def forward(self, u_k, q, du, periodic, tau):
        _check(_lib.tbs_net_forward(self._h, _ptr(u_k), _ptr(q), _dtype_code(u_k), _ptr(du), int(periodic), tau),
               "tbs_net_forward")

    def train_step(self, u_k, q, du_target, batch, periodic, tau, want_loss=True):
        loss = ctypes.c_float()
        _check(_lib.tbs_net_train_step(self._h, _ptr(u_k), _ptr(q), _ptr(du_target), batch, int(periodic), tau,
                                       ctypes.byref(loss) if want_loss else None), "tbs_net_train_step")
        return loss.value if want_loss else None

    def conv_layer(self, layer, mode, x, g, periodic, out):
        """mode 0: forward pre-activation; 1: data gradient; 2: weight+bias gradient (see tbs.h)."""
        _check(_lib.tbs_net_conv_layer(self._h, layer, mode, _ptr(x), _ptr(g), int(periodic), _ptr(out)),
               "tbs_net_conv_layer")

    def get_grad(self):
        import numpy as np
        w = np.zeros(NET_PARAMS, dtype=np.float32)
        _check(_lib.tbs_net_get_grad(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size),
               "tbs_net_get_grad")
        return w
