"""Python binding of libsmc2.so (include/smc2.h): argument marshalling only.

Every function below has the name of the C entry point it calls and forwards device pointers
of torch tensors plus the current HIP stream.  All arithmetic of the hot path runs in the
library's kernels; nothing here computes any part of it.  If the library is not built, loading
fails loudly: there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsmc2.so")

SMC2_OK, SMC2_E_INVALID_ARG, SMC2_E_UNSUPPORTED, SMC2_E_OUT_OF_MEMORY, SMC2_E_DEVICE, \
    SMC2_E_NONFINITE = range(6)
STATUS_NAMES = {0: "SMC2_OK", 1: "SMC2_E_INVALID_ARG", 2: "SMC2_E_UNSUPPORTED",
                3: "SMC2_E_OUT_OF_MEMORY", 4: "SMC2_E_DEVICE", 5: "SMC2_E_NONFINITE"}
LG1D, LG_DIAG, GROWTH, SV, LG1D_OPT, SIR = 0, 1, 2, 3, 4, 5
PRIOR_NORMAL, PRIOR_UNIFORM = 0, 1
FP64, MIXED = 0, 1
SYSTEMATIC, MULTINOMIAL = 0, 1


class SMC2Error(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__("%s failed with %s: %s" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


class smc2_model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d_x", ctypes.c_int32), ("d_y", ctypes.c_int32),
                ("D", ctypes.c_int32), ("prior_mu", ctypes.POINTER(ctypes.c_double)),
                ("prior_sd", ctypes.POINTER(ctypes.c_double)),
                ("prior_kind", ctypes.POINTER(ctypes.c_int32)),
                ("constants", ctypes.POINTER(ctypes.c_double))]


class smc2_pf_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("resampler", ctypes.c_int32),
                ("ess_frac", ctypes.c_double), ("ckpt_interval", ctypes.c_int32),
                ("want_grad", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("store_noise", ctypes.c_int32)]


class smc2_population(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("logpost", ctypes.c_void_p),
                ("grad_logpost", ctypes.c_void_p), ("loglik", ctypes.c_void_p),
                ("logw", ctypes.c_void_p)]


_lib = None

# (name, restype, argtypes) of every exported entry point of include/smc2.h
_VP, _I32, _U64, _D, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, \
    ctypes.c_size_t
_MP, _OP, _POP = ctypes.POINTER(smc2_model), ctypes.POINTER(smc2_pf_opts), \
    ctypes.POINTER(smc2_population)
SIGNATURES = [
    ("smc2_ctx_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int]),
    ("smc2_ctx_reserve", ctypes.c_int, [_VP, _MP, _OP, _I32, _I32, _I32, _VP, _I32, _SZ]),
    ("smc2_ctx_scratch_bytes", ctypes.c_int, [_MP, _OP, _I32, _I32, _I32, _I32,
                                              ctypes.POINTER(_SZ)]),
    ("smc2_ctx_destroy", None, [_VP]),
    ("smc2_last_error", ctypes.c_char_p, []),
    ("smc2_ctx_device_status", ctypes.c_int, [_VP, _VP]),
    ("smc2_pf_loglik_grad", ctypes.c_int, [_VP, _MP, _OP, _I32, _I32, _I32, _VP, _I32, _VP, _VP,
                                           _U64, _VP, _VP, _VP, _VP]),
    ("smc2_langevin_move", ctypes.c_int, [_VP, _MP, _I32, _I32, _D, _I32, _VP, _VP, _U64, _VP,
                                          _VP, _VP, _VP]),
    ("smc2_reweight_resample", ctypes.c_int, [_VP, _MP, _I32, _I32, _D, _I32, _POP, _POP, _VP,
                                              _I32, _U64, _VP, _I32, _VP, _VP, _VP, _VP, _VP,
                                              _VP]),
    ("smc2_reweight_resample_noalloc", ctypes.c_int, [_MP, _I32, _I32, _D, _I32, _POP, _POP,
                                                      _VP, _I32, _U64, _VP, _I32, _VP, _VP, _VP,
                                                      _VP, _VP, _VP, _VP]),
    ("smc2_prior_init", ctypes.c_int, [_VP, _MP, _I32, _I32, _U64, _VP, _VP]),
    ("smc2_pf_trace", ctypes.c_int, [_VP, _I32, _I32, _VP, _VP, _VP, _VP]),
    ("smc2_philox_probe", ctypes.c_int, [_I32, _VP, _VP, _U64, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("smc2_tile_info", ctypes.c_int, [_I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                      ctypes.POINTER(_I32)]),
    ("smc2_version", ctypes.c_char_p, []),
]


def lib():
    """Load libsmc2.so (raises if it is not built: the product path has no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsmc2.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status != SMC2_OK:
        raise SMC2Error(status, where, lib().smc2_last_error().decode())


def _ptr(t, dtype=None, name="tensor", numel=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL) that holds at least `numel`
    elements (the kernels index it by the sizes passed alongside, so a smaller buffer is refused
    here rather than read or written past its end)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements; the sizes need %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Model:
    """A smc2_model with its prior and constant arrays kept alive.  d_y is 1 for the SIR model
    and d_x otherwise; prior_kind (None: all normal) and constants (None: the model's defaults)
    are passed through as given."""

    def __init__(self, kind, d_x, D, prior_mu=None, prior_sd=None, prior_kind=None,
                 constants=None):
        self.kind, self.d_x, self.D = int(kind), int(d_x), int(D)
        self.d_y = 1 if self.kind == SIR else self.d_x
        self.prior_mu = np.ascontiguousarray(np.zeros(D) if prior_mu is None else prior_mu, np.float64)
        self.prior_sd = np.ascontiguousarray(np.ones(D) if prior_sd is None else prior_sd, np.float64)
        self.prior_kind = (None if prior_kind is None
                           else np.ascontiguousarray(prior_kind, np.int32))
        self.constants = None if constants is None else np.ascontiguousarray(constants, np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        self.c = smc2_model(self.kind, self.d_x, self.d_y, self.D,
                            self.prior_mu.ctypes.data_as(dp), self.prior_sd.ctypes.data_as(dp),
                            None if self.prior_kind is None else self.prior_kind.ctypes.data_as(ip),
                            None if self.constants is None else self.constants.ctypes.data_as(dp))

    @classmethod
    def from_workload(cls, w):
        return cls(w.kind, w.d, w.D, w.prior_mu, w.prior_sd, getattr(w, "prior_kind", None),
                   getattr(w, "constants", None))


def pf_opts(precision=FP64, resampler=SYSTEMATIC, ess_frac=0.5, ckpt_interval=0, want_grad=1,
            tile=0, persistent=0, store_noise=0):
    return smc2_pf_opts(int(precision), int(resampler), float(ess_frac), int(ckpt_interval),
                        int(want_grad), int(tile), int(persistent), int(store_noise))


# ---- entry points (same names as the C ABI) ----------------------------------------------------

def smc2_version():
    return lib().smc2_version().decode()


def smc2_ctx_create(device=0):
    h = ctypes.c_void_p()
    _check(lib().smc2_ctx_create(ctypes.byref(h), int(device)), "smc2_ctx_create")
    return h


def smc2_ctx_destroy(ctx):
    lib().smc2_ctx_destroy(ctx)


def smc2_ctx_reserve(ctx, model, opts, S, N, M, T_len, T_max, scratch_budget_bytes=0):
    T_len = np.ascontiguousarray(T_len, dtype=np.int32)
    _check(lib().smc2_ctx_reserve(ctx, ctypes.byref(model.c), ctypes.byref(opts), int(S), int(N),
                                  int(M), T_len.ctypes.data_as(ctypes.c_void_p), int(T_max),
                                  int(scratch_budget_bytes)), "smc2_ctx_reserve")


def smc2_ctx_scratch_bytes(model, opts, S, N, M, T_max):
    out = ctypes.c_size_t(0)
    _check(lib().smc2_ctx_scratch_bytes(ctypes.byref(model.c), ctypes.byref(opts), int(S), int(N),
                                        int(M), int(T_max), ctypes.byref(out)),
           "smc2_ctx_scratch_bytes")
    return out.value


def smc2_ctx_device_status(ctx, stream=None):
    return lib().smc2_ctx_device_status(ctx, _stream(stream))


def smc2_pf_loglik_grad(ctx, model, opts, S, N, M, T_len, T_max, theta, y, seed, iteration,
                        loglik, grad, stream=None):
    T_len = np.ascontiguousarray(T_len, dtype=np.int32)
    if T_len.size < int(S):
        raise ValueError("T_len holds %d lengths; S = %d" % (T_len.size, int(S)))
    SN, D = int(S) * int(N), int(model.c.D)
    _check(lib().smc2_pf_loglik_grad(
        ctx, ctypes.byref(model.c), ctypes.byref(opts), int(S), int(N), int(M),
        T_len.ctypes.data_as(ctypes.c_void_p), int(T_max),
        _ptr(theta, torch.float64, "theta", SN * D),
        _ptr(y, torch.float64, "y", int(S) * int(T_max) * int(model.c.d_y)), int(seed),
        _ptr(iteration, torch.int32, "iteration", 1), _ptr(loglik, torch.float64, "loglik", SN),
        _ptr(grad, torch.float64, "grad", SN * D), _stream(stream)), "smc2_pf_loglik_grad")


def smc2_langevin_move(ctx, model, S, N, gamma, random_walk, theta, grad_logpost, seed,
                       iteration, theta_new, p_prev, stream=None):
    n = int(S) * int(N) * int(model.c.D)
    _check(lib().smc2_langevin_move(
        ctx, ctypes.byref(model.c), int(S), int(N), float(gamma), int(random_walk),
        _ptr(theta, torch.float64, "theta", n),
        _ptr(grad_logpost, torch.float64, "grad_logpost", n),
        int(seed), _ptr(iteration, torch.int32, "iteration", 1),
        _ptr(theta_new, torch.float64, "theta_new", n), _ptr(p_prev, torch.float64, "p_prev", n),
        _stream(stream)), "smc2_langevin_move")


def population(theta, logpost, grad_logpost, loglik, logw):
    """A smc2_population over five float64 CUDA tensors (their sizes are kept with it and checked
    against S, N and D where it is used)."""
    pop = smc2_population(*[_ptr(t, torch.float64, n) for t, n in
                            ((theta, "theta"), (logpost, "logpost"),
                             (grad_logpost, "grad_logpost"), (loglik, "loglik"), (logw, "logw"))])
    pop.numels = dict(theta=theta.numel(), logpost=logpost.numel(),
                      grad_logpost=grad_logpost.numel(), loglik=loglik.numel(),
                      logw=logw.numel())
    return pop


def _check_population(pop, SN, D, name):
    need = dict(theta=SN * D, logpost=SN, grad_logpost=SN * D, loglik=SN, logw=SN)
    have = getattr(pop, "numels", None)
    if have is None:
        return
    for k, v in need.items():
        if have[k] < v:
            raise ValueError("%s.%s holds %d elements; the sizes need %d" % (name, k, have[k], v))


def smc2_reweight_resample(ctx, model, S, N, gamma, random_walk, cur, prev, p_prev,
                           first_iteration, seed, iteration, advance_iteration=0,
                           ancestors=None, ess=None, resampled=None, estimate=None,
                           recycle=None, stream=None):
    SN, D = int(S) * int(N), int(model.c.D)
    _check_population(cur, SN, D, "cur")
    if prev is not None and not first_iteration:
        _check_population(prev, SN, D, "prev")
    _check(lib().smc2_reweight_resample(
        ctx, ctypes.byref(model.c), int(S), int(N), float(gamma), int(random_walk),
        ctypes.byref(cur), None if prev is None else ctypes.byref(prev),
        _ptr(p_prev, torch.float64, "p_prev", None if first_iteration else SN * D),
        int(first_iteration), int(seed),
        _ptr(iteration, torch.int32, "iteration", 1), int(advance_iteration),
        _ptr(ancestors, torch.int32, "ancestors", SN), _ptr(ess, torch.float64, "ess", int(S)),
        _ptr(resampled, torch.int32, "resampled", int(S)),
        _ptr(estimate, torch.float64, "estimate", int(S) * 2 * D),
        _ptr(recycle, torch.float64, "recycle", int(S) * (1 + 4 * D)), _stream(stream)),
        "smc2_reweight_resample")


def smc2_reweight_resample_noalloc(model, S, N, gamma, random_walk, cur, prev, p_prev,
                                   first_iteration, seed, iteration, advance_iteration=0,
                                   ancestors=None, ess=None, resampled=None, estimate=None,
                                   recycle=None, status=None, stream=None):
    SN, D = int(S) * int(N), int(model.c.D)
    _check_population(cur, SN, D, "cur")
    if prev is not None and not first_iteration:
        _check_population(prev, SN, D, "prev")
    _check(lib().smc2_reweight_resample_noalloc(
        ctypes.byref(model.c), int(S), int(N), float(gamma), int(random_walk),
        ctypes.byref(cur), None if prev is None else ctypes.byref(prev),
        _ptr(p_prev, torch.float64, "p_prev", None if first_iteration else SN * D),
        int(first_iteration), int(seed),
        _ptr(iteration, torch.int32, "iteration", 1), int(advance_iteration),
        _ptr(ancestors, torch.int32, "ancestors", SN), _ptr(ess, torch.float64, "ess", int(S)),
        _ptr(resampled, torch.int32, "resampled", int(S)),
        _ptr(estimate, torch.float64, "estimate", int(S) * 2 * D),
        _ptr(recycle, torch.float64, "recycle", int(S) * (1 + 4 * D)),
        _ptr(status, torch.int32, "status", 1), _stream(stream)),
        "smc2_reweight_resample_noalloc")


def smc2_prior_init(ctx, model, S, N, seed, theta, stream=None):
    _check(lib().smc2_prior_init(ctx, ctypes.byref(model.c), int(S), int(N), int(seed),
                                 _ptr(theta, torch.float64, "theta",
                                      int(S) * int(N) * int(model.c.D)), _stream(stream)),
           "smc2_prior_init")


def smc2_pf_trace(ctx, s, i, T, M, stream=None, with_steps=False):
    """(flags [T], ancestors [T][M]) of item (s, i), and with with_steps the per-step log
    normalisers s_t [T] as a third element."""
    flags = np.zeros(max(T, 1), dtype=np.uint8)
    anc = np.full((max(T, 1), M), -1, dtype=np.int32)
    st = np.full(max(T, 1), np.nan) if with_steps else None
    _check(lib().smc2_pf_trace(ctx, int(s), int(i), flags.ctypes.data_as(ctypes.c_void_p),
                               anc.ctypes.data_as(ctypes.c_void_p),
                               None if st is None else st.ctypes.data_as(ctypes.c_void_p),
                               _stream(stream)), "smc2_pf_trace")
    if with_steps:
        return flags[:T], anc[:T], st[:T]
    return flags[:T], anc[:T]


def smc2_philox_probe(ctr, n, seed, stream=None):
    """ctr: uint32-valued int64 CUDA tensor [R][4] passed as int32 bits; n: [R]."""
    R = ctr.shape[0]
    dev = ctr.device
    out = torch.zeros((R, 4), dtype=torch.int32, device=dev)
    normals = torch.zeros(R, dtype=torch.float64, device=dev)
    uniforms = torch.zeros(R, dtype=torch.float64, device=dev)
    n32 = torch.zeros(R, dtype=torch.float32, device=dev)
    u32 = torch.zeros(R, dtype=torch.float32, device=dev)
    _check(lib().smc2_philox_probe(int(R), _ptr(ctr, torch.int32, "ctr", 4 * R),
                                   _ptr(n, torch.int32, "n", R), int(seed), _ptr(out), _ptr(normals),
                                   _ptr(uniforms), _ptr(n32), _ptr(u32), _stream(stream)),
           "smc2_philox_probe")
    return out, normals, uniforms, n32, u32


def smc2_tile_info(tile, d_x=1):
    mp, w, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().smc2_tile_info(int(tile), int(d_x), ctypes.byref(mp), ctypes.byref(w),
                                ctypes.byref(p)), "smc2_tile_info")
    return mp.value, w.value, p.value


# ---- conveniences over the entry points -----------------------------------------------------

class Context:
    """Owns an smc2_ctx and its reservation for one workload shape."""

    def __init__(self, model, opts, S, N, M, T_len, T_max, device=0, scratch_budget_bytes=0):
        self.model, self.opts = model, opts
        self.S, self.N, self.M = int(S), int(N), int(M)
        self.T_len = np.ascontiguousarray(T_len, dtype=np.int32)
        self.T_max = int(T_max)
        self.h = smc2_ctx_create(device)
        try:
            smc2_ctx_reserve(self.h, model, opts, S, N, M, self.T_len, T_max, scratch_budget_bytes)
        except Exception:
            smc2_ctx_destroy(self.h)
            self.h = None
            raise

    def close(self):
        if self.h is not None:
            smc2_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pf(self, theta, y, seed, iteration, loglik, grad, opts=None, stream=None):
        smc2_pf_loglik_grad(self.h, self.model, opts or self.opts, self.S, self.N, self.M,
                            self.T_len, self.T_max, theta, y, seed, iteration, loglik, grad,
                            stream)


class PFLogLik(torch.autograd.Function):
    """loglik(theta) of the CRN-PF as an autograd function: the forward runs the fused
    forward+adjoint kernel and keeps the gradient; the backward scales it by grad_output."""

    @staticmethod
    def forward(ctx_, theta, y, context, seed, iteration):
        if not context.opts.want_grad:
            raise ValueError("PFLogLik needs a context reserved with want_grad = 1: the backward "
                             "returns the gradient the forward kernel computes")
        S, N, D = context.S, context.N, context.model.D
        loglik = torch.empty((S, N), dtype=torch.float64, device=theta.device)
        grad = torch.empty((S, N, D), dtype=torch.float64, device=theta.device)
        context.pf(theta.detach().contiguous(), y.contiguous(), seed, iteration, loglik, grad)
        ctx_.save_for_backward(grad)
        return loglik

    @staticmethod
    def backward(ctx_, grad_out):
        (grad,) = ctx_.saved_tensors
        return grad_out.unsqueeze(-1) * grad, None, None, None, None
