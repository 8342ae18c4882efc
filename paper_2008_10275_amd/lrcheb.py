"""Python binding of the C ABI in include/lrcheb.h (argument marshalling only).

Every computation happens inside liblrcheb.so (HIP kernels for gfx950 plus the
host factorisation of the preconditioner).  If the library is missing this
module raises on load: there is no fallback.

Host arrays are NumPy float64 (column-major where the C ABI says so); device
buffers are torch CUDA tensors (row-major, contiguous rows with the given
leading dimension).  The CUDA stream of a context is torch's current stream at
creation time unless one is given.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrcheb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lrcheb.h")

LRC_OK, LRC_ENOTCONV, LRC_EINVAL, LRC_ENOMEM, LRC_EDEVICE = 0, 1, -1, -2, -3
LRC_ESINGULAR, LRC_EBREAKDOWN, LRC_ECALLBACK = -4, -5, -6
LRC_FP64, LRC_MIXED_FP32, LRC_MIXED_FP32_DIR, LRC_MIXED_BF16GRAM = 0, 1, 2, 3
LRC_SOLVER_CHEBYSHEV, LRC_SOLVER_GMREST = 0, 1
LRC_CHEB_DIRECTION, LRC_CHEB_THREE_TERM = 0, 1
LRC_SPMM_SKIP_EMPTY = 4
LRC_PREC_LU, LRC_PREC_ILU0 = 0, 1
LRC_INIT_ZERO, LRC_INIT_MEDIAN, LRC_INIT_GIVEN, LRC_INIT_GIVEN_JUDGED, LRC_INIT_NEWTON = 0, 1, 2, 3, 4


class LrcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lrcheb error {code}: {msg}")
        self.code = code


class lrc_opts(C.Structure):
    _fields_ = [("rank_cap", C.c_int), ("trunc_tol", C.c_double), ("res_tol", C.c_double),
                ("max_iter", C.c_int), ("restart", C.c_int), ("cheb_c", C.c_double),
                ("cheb_d", C.c_double), ("precision", C.c_int), ("refine_max", C.c_int),
                ("inner_tol", C.c_double), ("init", C.c_int), ("median_tol", C.c_double),
                ("verify_fp64", C.c_int), ("eager", C.c_int), ("inner_trunc_tol", C.c_double),
                ("res_ref", C.c_double), ("solver", C.c_int), ("recurrence", C.c_int)]


class lrc_info(C.Structure):
    _fields_ = [("rank", C.c_int), ("rank_x0", C.c_int), ("iters", C.c_int),
                ("prec_applies", C.c_int), ("refinements", C.c_int), ("median_iters", C.c_int),
                ("relres", C.c_double), ("relres_est", C.c_double),
                ("max_col_relres", C.c_double), ("seconds_setup", C.c_double),
                ("seconds_solve", C.c_double), ("info_flags", C.c_int), ("status", C.c_int),
                ("newton_steps", C.c_int), ("median_fallback_cols", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# int cb(void* user, int k, int stage, const double* x, double* const* val_out,
#        int* rB, double* BU, double* BV, double* bnorm)
LINEARIZE_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double),
                           C.POINTER(C.POINTER(C.c_double)), C.POINTER(C.c_int),
                           C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double))
MAX_RHS_RANK = 8

_P = C.c_void_p
_SIGS = {
    "lrc_opts_default": (None, [C.POINTER(lrc_opts)]),
    "lrc_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "lrc_destroy": (None, [_P]),
    "lrc_last_error": (C.c_char_p, [_P]),
    "lrc_set_stream": (C.c_int, [_P, _P]),
    "lrc_ops_create": (C.c_int, [_P, C.c_int64, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                 C.POINTER(_P), C.POINTER(_P)]),
    "lrc_ops_update_values": (C.c_int, [_P, C.c_int, _P]),
    "lrc_ops_destroy": (None, [_P]),
    "lrc_ops_spmm_dev": (C.c_int, [_P, C.c_int, C.c_int, _P, C.c_int, _P, C.c_int]),
    "lrc_ops_spmm_tune": (C.c_int, [_P, C.c_int, C.c_int, _P, _P]),
    "lrc_ops_spmm_shape_dev": (C.c_int, [_P, C.c_int, C.c_int, _P, C.c_int, _P, C.c_int, _P]),
    "lrc_prob_create": (C.c_int, [_P, C.c_int64, _P, C.c_int, _P, _P, _P, C.POINTER(_P)]),
    "lrc_prob_destroy": (None, [_P]),
    "lrc_prob_precondition": (C.c_int, [_P, _P, C.c_int, C.c_int]),
    "lrc_prob_spectrum": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lrc_prob_precond_stats": (C.c_int, [_P, _P]),
    "lrc_prob_prec_apply_dev": (C.c_int, [_P, C.c_int, C.c_int, _P, C.c_int, _P, C.c_int]),
    "lrc_solve": (C.c_int, [_P, C.POINTER(lrc_opts), C.c_int, _P, _P, _P,
                            C.POINTER(lrc_info)]),
    "lrc_solve_batched": (C.c_int, [_P, C.c_int, C.POINTER(lrc_opts), C.POINTER(lrc_info)]),
    "lrc_solve_x0_dev": (C.c_int, [_P, C.POINTER(lrc_opts), C.c_int, _P, C.c_int, _P, _P, C.c_int,
                                   C.POINTER(lrc_info)]),
    "lrc_get_solution": (C.c_int, [_P, C.POINTER(C.c_int), _P, _P, _P]),
    "lrc_residual": (C.c_int, [_P, C.POINTER(C.c_double), _P]),
    "lrc_truncate_dev": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int, _P, C.c_int, _P,
                                   _P, C.c_int, C.c_int, C.c_double, _P, C.c_int, _P, _P,
                                   C.c_int, C.POINTER(C.c_int)]),
    "lrc_truncate_noalloc_dev": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int, _P,
                                           C.c_int, _P, _P, C.c_int, C.c_int, C.c_double, _P,
                                           C.c_int, _P, _P, C.c_int, C.POINTER(C.c_int)]),
    "lrc_truncate_scaled_dev": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int, C.c_int, _P,
                                          C.c_int, _P, _P, C.c_int, _P, C.c_int, C.c_double, _P,
                                          C.c_int, _P, _P, C.c_int, C.POINTER(C.c_int)]),
    "lrc_mlp_create": (C.c_int, [_P, _P, _P, C.POINTER(_P)]),
    "lrc_mlp_destroy": (None, [_P]),
    "lrc_mlp_fit_scaling": (C.c_int, [_P, C.c_int, _P, _P]),
    "lrc_mlp_grad": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
    "lrc_mlp_train": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, C.c_float, C.c_float, C.c_float,
                                C.c_float, _P]),
    "lrc_mlp_predict": (C.c_int, [_P, C.c_int, _P, _P]),
    "lrc_mlp_get_params": (C.c_int, [_P, _P]),
    "lrc_profile_enable": (C.c_int, [C.c_int]),
    "lrc_profile_read": (C.c_int, [C.c_int, _P, _P, _P, _P]),
    "lrc_profile_class_name": (C.c_char_p, [C.c_int]),
    "lrc_theta_scheme": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, C.c_int, _P, C.c_int, _P, _P,
                                   _P, C.c_double, C.c_double, C.c_int, C.POINTER(lrc_opts),
                                   C.POINTER(_P), C.POINTER(lrc_info)]),
    "lrc_newton_subsets": (C.c_int, [_P, C.c_int64, _P, C.c_int, _P, _P, _P, LINEARIZE_FN, _P,
                                     C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(lrc_opts),
                                     C.POINTER(_P), C.POINTER(lrc_info), _P]),
}

_lib = None


def header_symbols():
    """Names of every function the public header declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lrc_[a-z_0-9]+)\s*\(", txt)) - {"lrc_linearize_fn"})


def load():
    """Load liblrcheb.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # One HIP runtime per process: torch ships its own libamdhip64 (soname
    # libamdhip64.so.7, requested as libamdhip64.so).  Loading torch first makes
    # the library's libamdhip64.so.7 dependency resolve to that same runtime, so
    # device pointers and streams from torch are valid inside the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a, order="F"):
    return np.require(np.asarray(a, dtype=np.float64), requirements=[order, "A", "O"])


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr())


def _check(ctx_handle, code):
    if code < 0:
        msg = load().lrc_last_error(ctx_handle)
        raise LrcError(code, msg.decode() if msg else "")
    return code


def default_opts(**kw):
    o = lrc_opts()
    load().lrc_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


# --------------------------------------------------------------------------- context
class Context:
    """lrc_create / lrc_destroy.  stream: an int hipStream_t (None: torch's current)."""

    def __init__(self, device=0, stream=None):
        lib = load()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.handle = C.c_void_p()
        code = lib.lrc_create(C.byref(self.handle), device, C.c_void_p(stream))
        if code != 0:
            raise LrcError(code, "lrc_create failed (no HIP device?)")
        self.device = device

    def close(self):
        if self.handle:
            load().lrc_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(self.handle, load().lrc_set_stream(self.handle, C.c_void_p(stream)))


class Operators:
    """lrc_ops_create from a list of SciPy CSR matrices."""

    def __init__(self, ctx, K):
        lib = load()
        self.ctx = ctx
        n = K[0].shape[0]
        self.n, self.q = n, len(K)
        self._keep = []
        rp, cl, vl = [], [], []
        for Ki in K:
            r = np.ascontiguousarray(Ki.indptr, dtype=np.int64)
            c = np.ascontiguousarray(Ki.indices, dtype=np.int32)
            v = np.ascontiguousarray(Ki.data, dtype=np.float64)
            self._keep += [r, c, v]
            rp.append(_ptr(r))
            cl.append(_ptr(c))
            vl.append(_ptr(v))
        arr = C.c_void_p * self.q
        self.nnz = [Ki.nnz for Ki in K]
        self.handle = C.c_void_p()
        _check(ctx.handle, lib.lrc_ops_create(ctx.handle, n, self.q, arr(*rp), arr(*cl),
                                              arr(*vl), C.byref(self.handle)))

    def spmm_tune(self, dtype, r):
        """lrc_ops_spmm_tune: (columns per lane, waves, grid cap), best us, default us."""
        cfg = np.zeros(3, dtype=np.int32)
        t = np.zeros(2)
        _check(self.ctx.handle, load().lrc_ops_spmm_tune(self.handle, int(dtype), int(r),
                                                         _ptr(cfg), _ptr(t)))
        return tuple(int(x) for x in cfg), float(t[0]), float(t[1])

    def update_values(self, i, val):
        v = np.ascontiguousarray(val, dtype=np.float64)
        _check(self.ctx.handle, load().lrc_ops_update_values(self.handle, i, _ptr(v)))

    def spmm_dev(self, U, W, r=None, skip_empty=False):
        """W (q*n x ldw tensor) = [K_0 U; ...; K_{q-1} U] for a row-major U tensor.
        skip_empty: rows of W whose operator row is empty are left untouched."""
        import torch
        dtype = (0 if U.dtype == torch.float64 else 1) | (LRC_SPMM_SKIP_EMPTY if skip_empty else 0)
        r = U.shape[1] if r is None else r
        _check(self.ctx.handle, load().lrc_ops_spmm_dev(self.handle, dtype, r, _dev_ptr(U),
                                                        U.stride(0), _dev_ptr(W), W.stride(0)))

    def spmm_shape_dev(self, U, W, shape, r=None):
        """spmm_dev with an explicit launch shape (columns per lane, waves, grid cap)."""
        import torch
        dtype = 0 if U.dtype == torch.float64 else 1
        r = U.shape[1] if r is None else r
        cfg = np.asarray(shape, dtype=np.int32)
        _check(self.ctx.handle, load().lrc_ops_spmm_shape_dev(
            self.handle, dtype, r, _dev_ptr(U), U.stride(0), _dev_ptr(W), W.stride(0), _ptr(cfg)))

    def close(self):
        if self.handle:
            load().lrc_ops_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """lrc_prob_create: one subset with table d (q x m) and F = FU diag(Fs) FV^T."""

    def __init__(self, ops, d, FU, FV, Fs=None, handle=None):
        self.ops = ops
        self.ctx = ops.ctx
        self.d = np.asarray(d, dtype=np.float64)
        self.m = self.d.shape[1]
        if handle is not None:
            self.handle = handle
            return
        FU = _f64(np.atleast_2d(FU.T).T if FU.ndim == 1 else FU)
        FV = _f64(np.atleast_2d(FV.T).T if FV.ndim == 1 else FV)
        dd = _f64(self.d)
        fs = None if Fs is None else _f64(Fs)
        self._keep = [FU, FV, dd, fs]
        self.handle = C.c_void_p()
        _check(self.ctx.handle, load().lrc_prob_create(ops.handle, self.m, _ptr(dd), FU.shape[1],
                                                       _ptr(FU), _ptr(fs), _ptr(FV),
                                                       C.byref(self.handle)))

    def precondition(self, dbar=None, leaf_size=0, kind=0):
        """lrc_prob_precondition; kind LRC_PREC_LU (exact) or LRC_PREC_ILU0."""
        db = None if dbar is None else _f64(dbar)
        _check(self.ctx.handle, load().lrc_prob_precondition(self.handle, _ptr(db), leaf_size,
                                                             kind))

    def spectrum(self):
        c, d = C.c_double(), C.c_double()
        _check(self.ctx.handle, load().lrc_prob_spectrum(self.handle, C.byref(c), C.byref(d)))
        return c.value, d.value

    def precond_stats(self):
        out = np.zeros(8)
        _check(self.ctx.handle, load().lrc_prob_precond_stats(self.handle, _ptr(out)))
        keys = ["supernodes", "levels_fwd", "levels_bwd", "max_front", "block_entries",
                "seconds_order", "seconds_factor", "seconds_upload"]
        return dict(zip(keys, out.tolist()))

    def prec_apply_dev(self, R, Z, k=None):
        import torch
        dtype = 0 if R.dtype == torch.float64 else 1
        k = R.shape[1] if k is None else k
        _check(self.ctx.handle, load().lrc_prob_prec_apply_dev(
            self.handle, dtype, k, _dev_ptr(R), R.stride(0), _dev_ptr(Z), Z.stride(0)))

    def solve(self, opts=None, X0=None, **kw):
        """lrc_solve; X0 = (U0, s0, V0) host arrays for LRC_INIT_GIVEN.  Returns
        (status, info dict)."""
        o = opts if opts is not None else default_opts(**kw)
        info = lrc_info()
        r0, U0, s0, V0 = 0, None, None, None
        if X0 is not None:
            U0, s0, V0 = _f64(X0[0]), None if X0[1] is None else _f64(X0[1]), _f64(X0[2])
            r0 = U0.shape[1]
        code = load().lrc_solve(self.handle, C.byref(o), r0, _ptr(U0), _ptr(s0), _ptr(V0),
                                C.byref(info))
        _check(self.ctx.handle, code)
        return code, info.as_dict()

    def solve_x0_dev(self, U0, V0, s0=None, opts=None, **kw):
        """lrc_solve_x0_dev: X0 = U0 diag(s0) V0^T from row-major fp64 device
        tensors (n x r0 and m x r0).  Returns (status, info dict)."""
        kw.setdefault("init", LRC_INIT_GIVEN)
        o = opts if opts is not None else default_opts(**kw)
        info = lrc_info()
        r0 = U0.shape[1]
        sv = None if s0 is None else _f64(s0)
        code = load().lrc_solve_x0_dev(self.handle, C.byref(o), r0, _dev_ptr(U0), U0.stride(0),
                                       _ptr(sv), _dev_ptr(V0), V0.stride(0), C.byref(info))
        _check(self.ctx.handle, code)
        return code, info.as_dict()

    def solution(self):
        """Factors (U, s, V) of X = U diag(s) V^T (host, the x0 term first)."""
        lib = load()
        r = C.c_int()
        _check(self.ctx.handle, lib.lrc_get_solution(self.handle, C.byref(r), None, None, None))
        U = np.zeros((self.ops.n, r.value), order="F")
        V = np.zeros((self.m, r.value), order="F")
        s = np.zeros(r.value)
        if r.value:
            _check(self.ctx.handle, lib.lrc_get_solution(self.handle, C.byref(r), _ptr(U),
                                                         _ptr(s), _ptr(V)))
        return U, s, V

    def residual(self):
        rr = C.c_double()
        col = np.zeros(self.m)
        _check(self.ctx.handle, load().lrc_residual(self.handle, C.byref(rr), _ptr(col)))
        return rr.value, col

    def close(self):
        if self.handle:
            load().lrc_prob_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(problems, opts=None, **kw):
    """lrc_solve_batched: all problems (one context, each preconditioned) in
    lockstep, one launch per step, each restart cycle replayed from captured
    HIP graphs.  Returns (worst status, [info dict per problem])."""
    if not problems:
        raise ValueError("solve_batched: no problems")
    o = opts if opts is not None else default_opts(**kw)
    K = len(problems)
    hs = (C.c_void_p * K)(*[p.handle.value for p in problems])
    infos = (lrc_info * K)()
    code = load().lrc_solve_batched(hs, K, C.byref(o), infos)
    _check(problems[0].ctx.handle, code)
    return code, [infos[k].as_dict() for k in range(K)]


class MLP:
    """Surrogate perceptron (lrc_mlp_*).  params: list [W1, b1, W2, b2, W3, b3]
    (W out x in, as in the oracle).  Data are fp64 torch tensors on the device:
    X (B x d0), T (B x d3)."""

    def __init__(self, ctx, params):
        self.ctx = ctx
        self.sizes = [params[0].shape[1], params[0].shape[0], params[2].shape[0],
                      params[4].shape[0]]
        self.shapes = [np.shape(p) for p in params]
        packed = np.concatenate([np.ravel(np.asarray(p, dtype=np.float64)) for p in params])
        packed = np.ascontiguousarray(packed, dtype=np.float32)
        sz = np.ascontiguousarray(self.sizes, dtype=np.int32)
        h = C.c_void_p()
        _check(ctx.handle, load().lrc_mlp_create(ctx.handle, _ptr(sz), _ptr(packed), C.byref(h)))
        self.handle = h
        self.np = packed.size

    def _unpack(self, flat):
        out, o = [], 0
        for sh in self.shapes:
            k = int(np.prod(sh))
            out.append(flat[o:o + k].reshape(sh).astype(np.float64))
            o += k
        return out

    @staticmethod
    def _dev(t):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("MLP data must be contiguous fp64 device tensors")
        return _dev_ptr(t)

    def fit_scaling(self, X, T):
        _check(self.ctx.handle, load().lrc_mlp_fit_scaling(self.handle, X.shape[0], self._dev(X),
                                                           self._dev(T)))

    def grad(self, X, T):
        """(loss, gradients as a list like params) of one forward/backward pass."""
        loss = C.c_float()
        g = np.zeros(self.np, dtype=np.float32)
        _check(self.ctx.handle, load().lrc_mlp_grad(self.handle, X.shape[0], self._dev(X),
                                                    self._dev(T), C.byref(loss), _ptr(g)))
        return float(loss.value), self._unpack(g)

    def train(self, X, T, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        hist = np.zeros(max(steps, 1), dtype=np.float32)
        _check(self.ctx.handle, load().lrc_mlp_train(self.handle, X.shape[0], self._dev(X),
                                                     self._dev(T), steps, lr, beta1, beta2, eps,
                                                     _ptr(hist)))
        return hist[:steps].astype(np.float64)

    def predict(self, X):
        import torch
        Y = torch.empty((X.shape[0], self.sizes[3]), dtype=torch.float64, device=X.device)
        _check(self.ctx.handle, load().lrc_mlp_predict(self.handle, X.shape[0], self._dev(X),
                                                       _dev_ptr(Y)))
        return Y

    def params(self):
        p = np.zeros(self.np, dtype=np.float32)
        _check(self.ctx.handle, load().lrc_mlp_get_params(self.handle, _ptr(p)))
        return self._unpack(p)

    def close(self):
        if getattr(self, "handle", None):
            load().lrc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(mode=1):
    """Per-kernel-class HIP event timing: 0 stop, 1 events, 2 events + work
    accounting (both 1 and 2 clear the record)."""
    code = load().lrc_profile_enable(int(mode))
    if code != 0:
        raise LrcError(code, "lrc_profile_enable: mode must be 0, 1 or 2")


def profile_read():
    """{class: dict(ms, count, work, unit)} of the launches recorded so far
    (unit: None, "B" or "flop")."""
    lib = load()
    n = lib.lrc_profile_read(0, None, None, None, None)
    ms = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int32)
    work = np.zeros(n)
    unit = np.zeros(n, dtype=np.int32)
    lib.lrc_profile_read(n, _ptr(ms), _ptr(cnt), _ptr(work), _ptr(unit))
    names = {0: None, 1: "B", 2: "flop"}
    return {lib.lrc_profile_class_name(i).decode(): dict(ms=float(ms[i]), count=int(cnt[i]),
                                                          work=float(work[i]),
                                                          unit=names[int(unit[i])])
            for i in range(n)}


def truncate_dev(ctx, A, c, B, rank_cap, tol, U, V, noalloc=False, bf16=False):
    """lrc_truncate_dev on row-major device tensors; returns (s, rank).
    noalloc=True calls lrc_truncate_noalloc_dev (fixed per-device scratch);
    bf16=True (fp32 tensors) takes the first CholeskyQR pass on bf16 Grams."""
    import torch
    dtype = 0 if A.dtype == torch.float64 else (2 if bf16 else 1)
    cc = _f64(np.ravel(c))
    n, k = A.shape[0], cc.size
    m = B.shape[0]
    if A.shape[1] < k or B.shape[1] < k:
        raise ValueError("A and B need at least len(c) columns")
    s = np.zeros(64)
    r = C.c_int()
    fn = load().lrc_truncate_noalloc_dev if noalloc else load().lrc_truncate_dev
    _check(ctx.handle, fn(ctx.handle, dtype, n, m, k, _dev_ptr(A), A.stride(0), _ptr(cc),
                          _dev_ptr(B), B.stride(0), rank_cap, tol, _dev_ptr(U), U.stride(0),
                          _ptr(s), _dev_ptr(V), V.stride(0), C.byref(r)))
    return s[:r.value].copy(), r.value


def truncate_scaled_dev(ctx, A, c, B, k1, w, rank_cap, tol, U, V):
    """lrc_truncate_scaled_dev: truncation of A diag(c) [B1 | diag(w) B2]^T
    (B1 = B[:, :k1]); w is an fp64 device tensor of m values.  Returns (s, rank)."""
    import torch
    dtype = 0 if A.dtype == torch.float64 else 1
    cc = _f64(np.ravel(c))
    n, k = A.shape[0], cc.size
    m = B.shape[0]
    if A.shape[1] < k or B.shape[1] < k:
        raise ValueError("A and B need at least len(c) columns")
    if w.dtype != torch.float64 or w.numel() != m:
        raise ValueError("w must hold m fp64 values")
    s = np.zeros(64)
    r = C.c_int()
    _check(ctx.handle, load().lrc_truncate_scaled_dev(
        ctx.handle, dtype, n, m, k, int(k1), _dev_ptr(A), A.stride(0), _ptr(cc), _dev_ptr(B),
        B.stride(0), _dev_ptr(w), rank_cap, tol, _dev_ptr(U), U.stride(0), _ptr(s), _dev_ptr(V),
        V.stride(0), C.byref(r)))
    return s[:r.value].copy(), r.value


def newton_subsets(ops, d, K, f=None, opts=None, sizes=None, linearize=None, x_init=None,
                   eps_newton=None, newton_max=8, picard=False, prec_kind=0, **kw):
    """lrc_newton_subsets (Algorithm 1).

    linearize(k, stage, x) -> (vals, BU, BV, bnorm): vals a list of q value
    arrays (None entries, or vals None, keep the current values), BU (n x rB)
    and BV (m_k x rB) the factors of the step's right-hand side at x (stage 0:
    B_k(x); stage 1: b 1^T), bnorm = ||b||.  Without a callback the operators
    are taken as linear and f is the load vector.  eps_newton defaults to
    10 median_tol ||f||.  Returns (status, [Problem], [info dict], sizes) with the
    subset sizes the library used."""
    lib = load()
    o = opts if opts is not None else default_opts(**kw)
    dd = _f64(d)
    ff = None if f is None else _f64(f)
    xi = None if x_init is None else _f64(x_init)
    sz = None if sizes is None else np.ascontiguousarray(sizes, dtype=np.int64)
    n = ops.n
    if eps_newton is None:
        if ff is None:
            raise ValueError("eps_newton is required with a callback")
        # ten times the median solve's relative accuracy: one Newton step per
        # subset on linear operators
        eps_newton = 10.0 * (o.median_tol if o.median_tol > 0 else 1e-6) * \
            float(np.linalg.norm(ff))
    sizes_out = np.zeros(K, dtype=np.int64)
    err = []

    def _cb(user, k, stage, xp, vals, rB, BU, BV, bnorm):
        try:
            x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            new_vals, bu, bv, bn = linearize(k, stage, x)
            if new_vals is not None:
                for i, v in enumerate(new_vals):
                    if v is None:
                        continue
                    dst = np.ctypeslib.as_array(vals[i], shape=(ops.nnz[i],))
                    dst[:] = v
            bu = np.asarray(bu, dtype=np.float64).reshape(n, -1)
            mk = int(sizes_out[k])
            bv = np.asarray(bv, dtype=np.float64).reshape(mk, -1)
            r = bu.shape[1]
            if r < 1 or r > MAX_RHS_RANK or bv.shape[1] != r:
                raise ValueError("right-hand side rank")
            np.ctypeslib.as_array(BU, shape=(MAX_RHS_RANK * n,))[:n * r] = bu.reshape(-1, order="F")
            np.ctypeslib.as_array(BV, shape=(MAX_RHS_RANK * mk,))[:mk * r] = \
                bv.reshape(-1, order="F")
            rB[0] = r
            bnorm[0] = float(bn)
            return 0
        except Exception as e:   # reported after the call
            err.append(e)
            return 1

    cb = LINEARIZE_FN(_cb) if linearize is not None else C.cast(None, LINEARIZE_FN)
    out = (C.c_void_p * K)()
    infos = (lrc_info * K)()
    if linearize is not None:
        # the callback needs the subset sizes before the library reports them
        m = dd.shape[1]
        sizes_out[:] = sz if sz is not None else [m // K] * (K - 1) + [m - (K - 1) * (m // K)]
    code = lib.lrc_newton_subsets(ops.handle, dd.shape[1], _ptr(dd), K, _ptr(sz), _ptr(ff),
                                  _ptr(xi), cb, None, float(eps_newton), int(newton_max),
                                  int(bool(picard)), int(prec_kind), C.byref(o), out, infos,
                                  _ptr(sizes_out))
    if err:
        raise err[0]
    _check(ops.ctx.handle, code)
    probs = []
    off = 0
    for k in range(K):
        p = Problem(ops, dd[:, off:off + int(sizes_out[k])], None, None,
                    handle=C.c_void_p(out[k]))
        probs.append(p)
        off += int(sizes_out[k])
    return code, probs, [infos[k].as_dict() for k in range(K)], [int(v) for v in sizes_out]


def theta_scheme(ops, M, d, b, theta, dt, X0=None, history="exact", opts=None, **kw):
    """lrc_theta_scheme: len(b) - 1 theta steps of M X' + L(X) = b(t) 1^T.
    M: scipy CSR mass matrix; b: list of load vectors b(t_0..t_w); X0 =
    (U0, s0, V0) host factors or None (zero).  Returns (status, Problem of the
    last step, [info dict per step])."""
    lib = load()
    o = opts if opts is not None else default_opts(**kw)
    dd = _f64(d)
    steps = len(b) - 1
    bb = np.asfortranarray(np.column_stack([np.asarray(v, dtype=np.float64) for v in b]))
    rp = np.ascontiguousarray(M.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(M.indices, dtype=np.int32)
    mv = np.ascontiguousarray(M.data, dtype=np.float64)
    r0, U0, s0, V0 = 0, None, None, None
    if X0 is not None:
        U0, s0, V0 = _f64(X0[0]), None if X0[1] is None else _f64(X0[1]), _f64(X0[2])
        r0 = U0.shape[1]
    out = C.c_void_p()
    infos = (lrc_info * steps)()
    code = lib.lrc_theta_scheme(ops.handle, _ptr(rp), _ptr(ci), _ptr(mv), dd.shape[1], _ptr(dd),
                                steps, _ptr(bb), r0, _ptr(U0), _ptr(s0), _ptr(V0), float(theta),
                                float(dt), {"exact": 0, "median": 1}[history], C.byref(o),
                                C.byref(out), infos)
    _check(ops.ctx.handle, code)
    p = Problem(ops, dd, None, None, handle=C.c_void_p(out.value))
    return code, p, [infos[k].as_dict() for k in range(steps)]
