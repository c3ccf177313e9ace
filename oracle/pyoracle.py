"""ctypes wrapper of the serial FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product package.  The oracle shares no code with the HIP path.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.cpp")

LG1D, LG_DIAG, GROWTH, SV, LG1D_OPT, SIR = 0, 1, 2, 3, 4, 5
PRIOR_KIND_NORMAL, PRIOR_KIND_UNIFORM = 0, 1
INIT_NORMAL, STEP_NORMAL, RESAMPLE_UNIFORM, PRIOR_NORMAL, MOVE_NORMAL, OUTER_RESAMPLE_UNIFORM = (
    1, 2, 3, 4, 5, 6)
SYSTEMATIC, MULTINOMIAL = 0, 1


def build(force=True):
    """Compile liboracle.so with g++ (serial, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                           "-Wall", "-Wextra", "-o", tmp, SRC_PATH])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d", ctypes.c_int32), ("D", ctypes.c_int32),
                ("prior_mu", ctypes.POINTER(ctypes.c_double)),
                ("prior_sd", ctypes.POINTER(ctypes.c_double)),
                ("prior_kind", ctypes.POINTER(ctypes.c_int32)),
                ("constants", ctypes.POINTER(ctypes.c_double))]


class _PFOpts(ctypes.Structure):
    _fields_ = [("resampler", ctypes.c_int32), ("ess_frac", ctypes.c_double)]


class _SMC2Opts(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
                ("series", ctypes.c_int32), ("gamma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("proposal", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _configure(ctypes.CDLL(LIB_PATH))
    return _lib


def build_variant(path, replacements):
    """Compile a copy of the oracle with each (old, new) source replacement applied (each old
    text must occur exactly once) into `path` and load it: tests plant mistakes this way to show
    that a pin catches them."""
    with open(SRC_PATH) as f:
        src = f.read()
    for old, new in replacements:
        if src.count(old) != 1:
            raise ValueError("replacement text must occur once: %r" % old)
        src = src.replace(old, new)
    cpp = path + ".cpp"
    with open(cpp, "w") as f:
        f.write(src)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                           "-I" + _HERE, "-o", path, cpp])
    return _configure(ctypes.CDLL(path))


def _configure(L):
    """Declare the argument and result types of every exported oracle function on L."""
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    mp = ctypes.POINTER(_Model)
    op = ctypes.POINTER(_PFOpts)
    u64, u32, i32, i64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int64
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_normal.argtypes = [u64, u32, u32, u32, u32]
    L.orc_normal.restype = ctypes.c_double
    L.orc_uniform.argtypes = [u64, u32, u32, u32, u32]
    L.orc_uniform.restype = ctypes.c_double
    L.orc_normals.argtypes = [u64, u32, u32, u32, u32, i64, dp]
    L.orc_uniforms.argtypes = [u64, u32, u32, u32, u32, i64, dp]
    L.orc_filter_normal.argtypes = [u64, u32, u32, u32, u32]
    L.orc_filter_normal.restype = ctypes.c_double
    L.orc_filter_uniform.argtypes = [u64, u32, u32, u32, u32, u32]
    L.orc_filter_uniform.restype = ctypes.c_double
    L.orc_resample_lower_bound.argtypes = [i32, dp, dp, ip]
    L.orc_pf.argtypes = [mp, op, dp, i32, dp, i32, u64, u32, u32, dp, dp, ip, u8p, dp]
    L.orc_pf.restype = ctypes.c_int
    L.orc_pf_complex_step.argtypes = [mp, op, dp, i32, dp, i32, u64, u32, u32, i32,
                                      ctypes.c_double, dp, dp, ip]
    L.orc_pf_complex_step.restype = ctypes.c_int
    L.orc_kalman.argtypes = [mp, dp, i32, dp, dp, dp]
    L.orc_kalman.restype = ctypes.c_int
    L.orc_log_prior.argtypes = [mp, dp, dp]
    L.orc_log_prior.restype = ctypes.c_double
    L.orc_langevin_move.argtypes = [i32, ctypes.c_double, dp, dp, dp, dp, dp]
    L.orc_random_walk_move.argtypes = [i32, ctypes.c_double, dp, dp, dp, dp]
    L.orc_lkernel_log_ratio.argtypes = [i32, ctypes.c_double, dp, dp, dp]
    L.orc_lkernel_log_ratio.restype = ctypes.c_double
    L.orc_realised_estimate.argtypes = [i32, i32, dp, dp, dp, dp]
    L.orc_realised_estimate.restype = ctypes.c_double
    L.orc_recycle.argtypes = [i32, i32, dp, dp, dp]
    L.orc_smc2_run.argtypes = [mp, op, ctypes.POINTER(_SMC2Opts), i32, dp, dp, dp, dp, dp, dp,
                               ip, ip, dp, dp]
    L.orc_smc2_run.restype = ctypes.c_int
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Model:
    """Model description for the oracle: kind, state dim d, parameter dim D, independent priors
    (normal by default; prior_kind[p] = PRIOR_KIND_UNIFORM reads prior_mu[p], prior_sd[p] as the
    bounds) and the model constants (None: the model's defaults)."""

    def __init__(self, kind, d, D, prior_mu=None, prior_sd=None, prior_kind=None,
                 constants=None):
        self.kind, self.d, self.D = int(kind), int(d), int(D)
        self.dy = 1 if self.kind == SIR else self.d
        self.prior_mu = _f64(np.zeros(D) if prior_mu is None else prior_mu)
        self.prior_sd = _f64(np.ones(D) if prior_sd is None else prior_sd)
        self.prior_kind = (None if prior_kind is None
                           else np.ascontiguousarray(prior_kind, dtype=np.int32))
        self.constants = None if constants is None else _f64(constants)
        self._s = _Model(self.kind, self.d, self.D, _dp(self.prior_mu), _dp(self.prior_sd),
                         _ip(self.prior_kind), _dp(self.constants))

    @property
    def ref(self):
        return ctypes.byref(self._s)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p),
                            out.ctypes.data_as(u32p))
    return out


def c3(k, stream):
    return ((int(k) << 8) | int(stream)) & 0xFFFFFFFF


def normals(seed, c0, c2, c3_, first, count):
    out = np.empty(int(count))
    lib().orc_normals(seed, c0, c2, c3_, first, int(count), _dp(out))
    return out


def uniforms(seed, c0, c2, c3_, first, count):
    out = np.empty(int(count))
    lib().orc_uniforms(seed, c0, c2, c3_, first, int(count), _dp(out))
    return out


def resample_lower_bound(w, u, L=None):
    w, u = _f64(w), _f64(u)
    a = np.empty(len(w), dtype=np.int32)
    (L or lib()).orc_resample_lower_bound(len(w), _dp(w), _dp(u), _ip(a))
    return a


def pf(model, theta, y, M, seed, k, filter_id, resampler=SYSTEMATIC, ess_frac=0.5,
       want_grad=True, want_trace=False, L=None):
    """Run the oracle CRN-PF (of the library L, default the oracle itself).  Returns
    dict(loglik, grad, ancestors, flags, s)."""
    theta = _f64(theta)
    y = _f64(y).reshape(-1)
    T = len(y) // model.dy if model.dy else 0
    opts = _PFOpts(int(resampler), float(ess_frac))
    ll = ctypes.c_double(0.0)
    grad = np.zeros(model.D) if want_grad else None
    anc = np.empty((T, M), dtype=np.int32) if want_trace else None
    flags = np.empty(T, dtype=np.uint8) if want_trace else None
    s = np.empty(T) if want_trace else None
    rc = (L or lib()).orc_pf(model.ref, ctypes.byref(opts), _dp(theta), T, _dp(y), int(M), int(seed),
                      int(k), int(filter_id), ctypes.byref(ll), _dp(grad), _ip(anc),
                      None if flags is None else flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                      _dp(s))
    if rc != 0:
        raise ValueError("oracle pf rejected its arguments")
    return dict(loglik=ll.value, grad=grad, ancestors=anc, flags=flags, s=s)


def pf_complex_step(model, theta, y, M, seed, k, filter_id, p, h=1e-30, resampler=SYSTEMATIC,
                    ess_frac=0.5):
    theta = _f64(theta)
    y = _f64(y).reshape(-1)
    T = len(y) // model.dy
    opts = _PFOpts(int(resampler), float(ess_frac))
    ll = ctypes.c_double(0.0)
    dl = ctypes.c_double(0.0)
    anc = np.empty((T, M), dtype=np.int32)
    rc = lib().orc_pf_complex_step(model.ref, ctypes.byref(opts), _dp(theta), T, _dp(y), int(M),
                                   int(seed), int(k), int(filter_id), int(p), float(h),
                                   ctypes.byref(ll), ctypes.byref(dl), _ip(anc))
    if rc != 0:
        raise ValueError("oracle complex step rejected its arguments")
    return ll.value, dl.value, anc


def kalman(model, theta, y):
    theta = _f64(theta)
    y = _f64(y).reshape(-1)
    T = len(y) // model.dy
    ll = ctypes.c_double(0.0)
    grad = np.zeros(model.D)
    rc = lib().orc_kalman(model.ref, _dp(theta), T, _dp(y), ctypes.byref(ll), _dp(grad))
    if rc != 0:
        raise ValueError("oracle kalman rejected its arguments")
    return ll.value, grad


def log_prior(model, theta):
    theta = _f64(theta)
    g = np.zeros(model.D)
    v = lib().orc_log_prior(model.ref, _dp(theta), _dp(g))
    return v, g


def langevin_move(gamma, theta, grad_logpost, xi):
    theta, g, xi = _f64(theta), _f64(grad_logpost), _f64(xi)
    D = len(theta)
    tn, pp = np.zeros(D), np.zeros(D)
    lib().orc_langevin_move(D, float(gamma), _dp(theta), _dp(g), _dp(xi), _dp(tn), _dp(pp))
    return tn, pp


def random_walk_move(gamma, theta, xi):
    theta, xi = _f64(theta), _f64(xi)
    D = len(theta)
    tn, pp = np.zeros(D), np.zeros(D)
    lib().orc_random_walk_move(D, float(gamma), _dp(theta), _dp(xi), _dp(tn), _dp(pp))
    return tn, pp


def lkernel_log_ratio(gamma, grad_prev, grad_new, p_prev):
    gp, gn, pp = _f64(grad_prev), _f64(grad_new), _f64(p_prev)
    return lib().orc_lkernel_log_ratio(len(gp), float(gamma), _dp(gp), _dp(gn), _dp(pp))


def realised_estimate(logw, theta):
    """(mean [D], second moment [D], recycling weight l) of a weighted sample population."""
    logw, theta = _f64(logw), _f64(theta)
    N, D = theta.shape
    mean, second = np.zeros(D), np.zeros(D)
    l = lib().orc_realised_estimate(N, D, _dp(logw), _dp(theta), _dp(mean), _dp(second))
    return mean, second, l


def recycle(l, est):
    """Recycled estimate over iterations: l [K], est [K][D] -> [D]."""
    l, est = _f64(l), _f64(est)
    K, D = est.shape
    out = np.zeros(D)
    lib().orc_recycle(K, D, _dp(l), _dp(est), _dp(out))
    return out


def smc2_run(model, y, N, M, K, gamma, seed, series=0, resampler=SYSTEMATIC, ess_frac=0.5,
             proposal=1):
    """Full oracle SMC^2 run on one series; returns the per-iteration records."""
    y = _f64(y).reshape(-1)
    T = len(y) // model.dy
    D = model.D
    opts = _PFOpts(int(resampler), float(ess_frac))
    so = _SMC2Opts(int(N), int(M), int(K), int(series), float(gamma), int(seed), int(proposal))
    rec = dict(theta=np.zeros((K, N, D)), loglik=np.zeros((K, N)), grad=np.zeros((K, N, D)),
               logw=np.zeros((K, N)), ess=np.zeros(K), resampled=np.zeros(K, dtype=np.int32),
               anc=np.zeros((K, N), dtype=np.int32), theta_out=np.zeros((N, D)),
               logw_out=np.zeros(N))
    rc = lib().orc_smc2_run(model.ref, ctypes.byref(opts), ctypes.byref(so), T, _dp(y),
                            _dp(rec["theta"]), _dp(rec["loglik"]), _dp(rec["grad"]),
                            _dp(rec["logw"]), _dp(rec["ess"]), _ip(rec["resampled"]),
                            _ip(rec["anc"]), _dp(rec["theta_out"]), _dp(rec["logw_out"]))
    if rc != 0:
        raise ValueError("oracle smc2 rejected its arguments")
    return rec
