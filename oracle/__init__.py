"""FP64 CPU oracle of the independent-ensemble bootstrap particle filter.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product library (``paper_1407_8071_amd``) never imports, links or runs it,
and it imports nothing from the product library.

The arithmetic lives in ``pf_oracle.c`` (plain C, FP64, single thread); this
module builds it with gcc, loads it with ctypes and wraps each step of
Algorithm 1 (Sec. 2.3) with numpy arrays.  Particle arrays here are
``[N, dx]`` float64 (particle-major).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KINDS = {"ou1d": 0, "lorenz63": 1, "fhn": 2, "fhn_paper": 3}
P_INIT, P_PROP, P_RESAMPLE, P_TRUTH_INIT, P_TRUTH_NOISE, P_OBS_NOISE, P_TRAIN, P_CONFIG = range(1, 9)
TRUTH_STREAM = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile pf_oracle.c into liboracle.so (plain gcc -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("dx", C.c_int), ("J", C.c_int), ("S", C.c_int),
        ("h", C.c_double), ("p", C.c_double * 4), ("sd", C.c_double * 2),
        ("dy", C.c_int), ("obs_idx", C.POINTER(C.c_int)), ("obs_var", C.c_double),
        ("prior_mean", C.POINTER(C.c_double)), ("prior_sd", C.POINTER(C.c_double)),
        ("q", C.c_double * 8),
    ]


_lib = None

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_U32 = C.POINTER(C.c_uint32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "pf_oracle.h"))):
            build(force=True)
        L = C.CDLL(_LIB)
        M = C.POINTER(_Model)
        sig = {
            "or_key": (None, [C.c_uint64, _U32]),
            "or_philox4x32_10": (None, [_U32, _U32, _U32]),
            "or_u01": (C.c_double, [C.c_uint32]),
            "or_normals4": (None, [_U32, _U32, _D]),
            "or_philox_stream": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, _U32]),
            "or_normal_stream": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, _D]),
            "or_drift": (None, [M, _D, _D]),
            "or_laplacian": (None, [C.c_int, _D, _D]),
            "or_step_noise": (None, [M, _U32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _D]),
            "or_em_step": (None, [M, _D, _D, _D]),
            "or_prior_draw": (None, [M, _U32, C.c_uint32, C.c_uint32, C.c_uint32, _D]),
            "or_loglik": (C.c_double, [M, _D, _D]),
            "or_init": (None, [M, C.c_uint64, C.c_uint32, C.c_int, _D]),
            "or_propagate": (None, [M, C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D]),
            "or_propagate_particle": (None, [M, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, _D]),
            "or_weights": (None, [M, C.c_int, _D, _D, _D]),
            "or_normalise": (C.c_int, [C.c_int, _D, _D, _D, _D]),
            "or_ess": (C.c_double, [C.c_int, _D]),
            "or_cdf": (None, [C.c_int, _D, C.c_double, C.c_int, _D]),
            "or_sorted_uniforms": (None, [C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D]),
            "or_ancestors": (None, [C.c_int, _D, _D, _I32]),
            "or_gather": (None, [C.c_int, C.c_int, _D, _I32, _D]),
            "or_mean": (None, [C.c_int, C.c_int, _D, _D]),
            "or_weighted_mean": (None, [C.c_int, C.c_int, _D, _D, C.c_double, _D]),
            "or_filter_interval": (C.c_int, [M, C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D, _D,
                                             _D, _D, _I32, _D, _D, _D]),
            "or_run_ensemble": (None, [M, C.c_uint64, C.c_int, C.c_int, C.c_int, _D, _D, _D, _D, _D]),
            "or_systematic_uniforms": (None, [C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D]),
            "or_stratified_uniforms": (None, [C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D]),
            "or_residual_ancestors": (None, [C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D,
                                             C.c_double, C.c_int, _I32]),
            "or_resample_scheme": (None, [C.c_int, C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D,
                                          _I32]),
            "or_apf_interval": (C.c_int, [M, C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D, _D,
                                          _D, _D, C.c_int, _D, _I32, _D, _D]),
            "or_fhnp_region": (C.c_int, [M, _D, _I32]),
            "or_fhnp_step": (C.c_int, [M, _U32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                       _D, _D]),
            "or_transition": (None, [M, _U32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _D,
                                     _D]),
            "or_filter_interval_sched": (C.c_int, [M, C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D,
                                                   _D, _D, _D, C.c_int, C.c_double, _D, _I32, _D,
                                                   _D, _D, C.POINTER(C.c_int)]),
            "or_simulate": (None, [M, C.c_uint64, C.c_int, _D, _D]),
            "or_kalman_ou": (C.c_double, [M, C.c_int, _D, _D, _D]),
            "or_mlp_nparams": (C.c_int, [C.c_int, C.c_int]),
            "or_bf16": (C.c_double, [C.c_double]),
            "or_mlp_forward": (None, [C.c_int, C.c_int, _D, _D, _D, _D, _D, C.c_int]),
            "or_mlp_backward": (None, [C.c_int, C.c_int, _D, _D, _D, _D]),
            "or_mlp_loss_grad": (C.c_double, [C.c_int, C.c_int, _D, C.c_int, _D, _D, _D]),
            "or_nearest_obs": (None, [M, _I32]),
            "or_fhn_features": (None, [M, _D, _D, _I32, C.c_int, C.c_int, _D]),
            "or_ou_features": (None, [M, _D, _D, C.c_int, _D]),
            "or_propagate_learned": (None, [M, _D, C.c_uint64, C.c_uint32, C.c_int, C.c_int, _D,
                                            _D, _D, C.c_int]),
            "or_propagate_learned_particle": (C.c_double, [M, _D, C.c_uint64, C.c_uint32,
                                                           C.c_uint32, C.c_int, _D, _D, C.c_int]),
            "or_filter_interval_learned": (C.c_int, [M, _D, C.c_uint64, C.c_uint32, C.c_int,
                                                     C.c_int, _D, _D, _D, _D, _I32, _D, _D, _D,
                                                     C.c_int]),
            "or_run_ensemble_learned": (None, [M, _D, C.c_uint64, C.c_int, C.c_int, C.c_int, _D,
                                               _D, _D, _D, _D, C.c_int]),
            "or_ou_optimal_u": (C.c_double, [M, C.c_double, C.c_double, C.c_int]),
            "or_train_run": (None, [M, C.c_uint64, C.c_uint32, C.c_int, _D]),
            "or_train_trajectory": (None, [M, C.c_uint64, C.c_uint32, _D, _D, _D, _D]),
            "or_train_tile": (None, [M, C.c_uint64, C.c_int, C.c_int, C.c_uint32,
                                     C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "or_adam_step": (None, [C.c_int, _D, _D, _D, _D, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _i32(a):
    return a.ctypes.data_as(_I32) if a is not None else None


def _u32(a):
    return a.ctypes.data_as(_U32) if a is not None else None


class Model:
    """A state-space model (tau_0, tau_t, g_t) of Sec. 2.2 for the oracle.

    ``spec`` is a plain dict: kind ('ou1d' | 'lorenz63' | 'fhn'), dx, J, S, h,
    params (4 numbers), noise_sd (2), obs_idx, obs_var, prior_mean, prior_sd.
    """

    def __init__(self, spec: dict):
        self.spec = dict(spec)
        self.kind = spec["kind"]
        self.dx = int(spec["dx"])
        self.J = int(spec.get("J", 0))
        self.S = int(spec["S"])
        self.obs_idx = np.ascontiguousarray(spec["obs_idx"], dtype=np.int32)
        self.dy = int(self.obs_idx.size)
        self.prior_mean = np.ascontiguousarray(spec["prior_mean"], dtype=np.float64)
        self.prior_sd = np.ascontiguousarray(spec["prior_sd"], dtype=np.float64)
        assert self.prior_mean.size == self.dx and self.prior_sd.size == self.dx
        p = list(spec["params"]) + [0.0] * (4 - len(spec["params"]))
        sd = list(spec["noise_sd"]) + [0.0] * (2 - len(spec["noise_sd"]))
        q = list(spec.get("params_ext", ())) + [0.0] * (8 - len(spec.get("params_ext", ())))
        self.c = _Model(
            KINDS[self.kind], self.dx, self.J, self.S, float(spec["h"]),
            (C.c_double * 4)(*p), (C.c_double * 2)(*sd), self.dy,
            self.obs_idx.ctypes.data_as(C.POINTER(C.c_int)), float(spec["obs_var"]),
            _d(self.prior_mean), _d(self.prior_sd), (C.c_double * 8)(*q))

    @property
    def ref(self):
        return C.byref(self.c)


# ---------------------------------------------------------------- RNG ---------
def key(seed: int) -> np.ndarray:
    k = np.zeros(2, np.uint32)
    lib().or_key(C.c_uint64(seed), _u32(k))
    return k


def philox(ctr, k) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    kk = np.ascontiguousarray(k, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_u32(c), _u32(kk), _u32(out))
    return out


def u01(x: int) -> float:
    return lib().or_u01(C.c_uint32(x))


def normals4(ctr, k) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    kk = np.ascontiguousarray(k, dtype=np.uint32)
    z = np.zeros(4)
    lib().or_normals4(_u32(c), _u32(kk), _d(z))
    return z


def philox_stream(seed, c1, c2, c3, n) -> np.ndarray:
    out = np.zeros(n, np.uint32)
    lib().or_philox_stream(C.c_uint64(seed), c1, c2, c3, n, _u32(out))
    return out


def normal_stream(seed, c1, c2, c3, n) -> np.ndarray:
    out = np.zeros(n)
    lib().or_normal_stream(C.c_uint64(seed), c1, c2, c3, n, _d(out))
    return out


# ---------------------------------------------------------------- model -------
def drift(m: Model, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros(m.dx)
    lib().or_drift(m.ref, _d(x), _d(f))
    return f


def laplacian(v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    J = v.shape[0]
    out = np.zeros_like(v)
    lib().or_laplacian(J, _d(v), _d(out))
    return out


def step_noise(m: Model, seed, purpose, c0, c1, n) -> np.ndarray:
    z = np.zeros(m.dx)
    lib().or_step_noise(m.ref, _u32(key(seed)), purpose, c0, c1, n, _d(z))
    return z


def em_step(m: Model, x, z) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    xo = np.zeros(m.dx)
    lib().or_em_step(m.ref, _d(x), _d(z), _d(xo))
    return xo


def loglik(m: Model, x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().or_loglik(m.ref, _d(x), _d(y))


# ---------------------------------------------------------------- filter ------
def init(m: Model, seed, filt, N) -> np.ndarray:
    X = np.zeros((N, m.dx))
    lib().or_init(m.ref, C.c_uint64(seed), filt, N, _d(X))
    return X


def prior_particle(m: Model, seed, filt, index) -> np.ndarray:
    """The prior draw x_0 of particle `index` of filter `filt` (Philox counter
    word 0 = index), as or_init draws it."""
    x = np.zeros(m.dx)
    lib().or_prior_draw(m.ref, _u32(key(seed)), P_INIT, index, filt, _d(x))
    return x


def propagate(m: Model, seed, filt, t, X) -> np.ndarray:
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    lib().or_propagate(m.ref, C.c_uint64(seed), filt, X.shape[0], t, _d(X))
    return X


def propagate_particle(m: Model, seed, filt, index, t, x) -> np.ndarray:
    """Interval t of one particle with Philox counter word 0 = index."""
    x = np.array(x, dtype=np.float64, copy=True)
    lib().or_propagate_particle(m.ref, C.c_uint64(seed), filt, index, t, _d(x))
    return x


def weights(m: Model, X, y) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    lw = np.zeros(X.shape[0])
    lib().or_weights(m.ref, X.shape[0], _d(X), _d(y), _d(lw))
    return lw


def normalise(lw):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    mx, W, s2 = C.c_double(), C.c_double(), C.c_double()
    deg = lib().or_normalise(lw.size, _d(lw), C.byref(mx), C.byref(W), C.byref(s2))
    return mx.value, W.value, s2.value, bool(deg)


def ess(lw) -> float:
    """Effective sample size (sum w)^2 / sum w^2 of the weights exp(lw)."""
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    return float(lib().or_ess(lw.size, _d(lw)))


def cdf(lw, mx, degenerate=False) -> np.ndarray:
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    out = np.zeros(lw.size)
    lib().or_cdf(lw.size, _d(lw), mx, int(degenerate), _d(out))
    return out


def sorted_uniforms(seed, filt, t, N) -> np.ndarray:
    U = np.zeros(N)
    lib().or_sorted_uniforms(C.c_uint64(seed), filt, t, N, _d(U))
    return U


def ancestors(Cdf, U) -> np.ndarray:
    Cdf = np.ascontiguousarray(Cdf, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    A = np.zeros(Cdf.size, np.int32)
    lib().or_ancestors(Cdf.size, _d(Cdf), _d(U), _i32(A))
    return A


def resample(seed, filt, t, lw):
    """Normalise + CDF + sorted uniforms + ancestor search (steps 2a-2b)."""
    mx, W, s2, deg = normalise(lw)
    Cdf = cdf(lw, mx, deg)
    U = sorted_uniforms(seed, filt, t, len(lw))
    return ancestors(Cdf, U), Cdf, U, (mx, W, s2, deg)


# resampling schemes (Sec. 2.3): multinomial, systematic, stratified, residual
SCHEMES = {"multinomial": 0, "systematic": 1, "stratified": 2, "residual": 3}


def systematic_uniforms(seed, filt, t, N) -> np.ndarray:
    U = np.zeros(N)
    lib().or_systematic_uniforms(C.c_uint64(seed), filt, t, N, _d(U))
    return U


def stratified_uniforms(seed, filt, t, N) -> np.ndarray:
    U = np.zeros(N)
    lib().or_stratified_uniforms(C.c_uint64(seed), filt, t, N, _d(U))
    return U


def resample_scheme(scheme, seed, filt, t, lw) -> np.ndarray:
    """Ancestors of the log-weights lw by `scheme` (name or number)."""
    sc = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    A = np.zeros(lw.size, np.int32)
    lib().or_resample_scheme(sc, C.c_uint64(seed), filt, t, lw.size, _d(lw), _i32(A))
    return A


def filter_interval_sched(m: "Model", seed, filt, t, X, lwc, y, logZ=0.0, scheme=0,
                          ess_threshold=0.0):
    """One interval with a resampling scheme and the ESS-triggered schedule
    (carried log-weights lwc, normalised to mean weight 1)."""
    sc = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    lwc = np.array(lwc, dtype=np.float64, copy=True)
    y = np.ascontiguousarray(y, dtype=np.float64)
    N = X.shape[0]
    lz = C.c_double(logZ)
    lw = np.zeros(N)
    A = np.zeros(N, np.int32)
    me = np.zeros(m.dx)
    mw = np.zeros(m.dx)
    ess = C.c_double()
    rs = C.c_int()
    deg = lib().or_filter_interval_sched(m.ref, C.c_uint64(seed), filt, N, t, _d(X), _d(lwc),
                                         _d(y), C.byref(lz), sc, float(ess_threshold), _d(lw),
                                         _i32(A), _d(me), _d(mw), C.byref(ess), C.byref(rs))
    return dict(X=X, lwc=lwc, lw=lw, A=A, mean_est=me, mean_w=mw, logZ=lz.value,
                ess=ess.value, resampled=bool(rs.value), degenerate=bool(deg))


def apf_interval(m: "Model", seed, filt, t, X, lwc, y, logZ=0.0, scheme=0):
    """One auxiliary-particle-filter interval (pilot, first-stage resampling,
    propagation, second-stage weights carried in lwc)."""
    sc = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    lwc = np.array(lwc, dtype=np.float64, copy=True)
    y = np.ascontiguousarray(y, dtype=np.float64)
    N = X.shape[0]
    lz = C.c_double(logZ)
    lw = np.zeros(N)
    A = np.zeros(N, np.int32)
    mw = np.zeros(m.dx)
    ess = C.c_double()
    deg = lib().or_apf_interval(m.ref, C.c_uint64(seed), filt, N, t, _d(X), _d(lwc), _d(y),
                                C.byref(lz), sc, _d(lw), _i32(A), _d(mw), C.byref(ess))
    return dict(X=X, lwc=lwc, lw=lw, A=A, mean_w=mw, logZ=lz.value, ess=ess.value,
                degenerate=bool(deg))


def fhnp_region(m: "Model", U):
    """Stimulus region of the paper's network from the U plane: (count, mask)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    reg = np.zeros(U.size, np.int32)
    c = lib().or_fhnp_region(m.ref, _d(U), _i32(reg))
    return int(c), reg.astype(bool)


def fhnp_step(m: "Model", seed, purpose, c0, c1, n, x):
    """One step of the paper's network: (next state, event centre or -1)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    xo = np.zeros_like(x)
    ev = lib().or_fhnp_step(m.ref, _u32(key(seed)), purpose, c0, c1, n, _d(x), _d(xo))
    return xo, int(ev)


def mean(X) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.zeros(X.shape[1])
    lib().or_mean(X.shape[0], X.shape[1], _d(X), _d(out))
    return out


def weighted_mean(X, lw, mx) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    out = np.zeros(X.shape[1])
    lib().or_weighted_mean(X.shape[0], X.shape[1], _d(X), _d(lw), mx, _d(out))
    return out


def filter_interval(m: Model, seed, filt, t, X, y, logZ=0.0):
    """One full interval of Algorithm 1 for one filter.  Returns a dict."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    y = np.ascontiguousarray(y, dtype=np.float64)
    N = X.shape[0]
    lz = C.c_double(logZ)
    lw = np.zeros(N)
    A = np.zeros(N, np.int32)
    mp = np.zeros(m.dx)
    mw = np.zeros(m.dx)
    ess = C.c_double()
    deg = lib().or_filter_interval(m.ref, C.c_uint64(seed), filt, N, t, _d(X), _d(y), C.byref(lz),
                                   _d(lw), _i32(A), _d(mp), _d(mw), C.byref(ess))
    return dict(X=X, lw=lw, A=A, mean_post=mp, mean_w=mw, logZ=lz.value, ess=ess.value,
                degenerate=bool(deg))


def run_ensemble(m: Model, seed, M, N, y):
    """Definition 3 over y[T, dy]: returns est[T,dx], est_w[T,dx], logZ[M], ess[T]."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    T = y.shape[0]
    est = np.zeros((T, m.dx))
    est_w = np.zeros((T, m.dx))
    logZ = np.zeros(M)
    ess = np.zeros(T)
    lib().or_run_ensemble(m.ref, C.c_uint64(seed), M, N, T, _d(y), _d(est), _d(est_w), _d(logZ),
                          _d(ess))
    return est, est_w, logZ, ess


def simulate(m: Model, seed, T):
    """Truth x_true[T+1, dx] and observations y[T, dy] from the truth stream."""
    xt = np.zeros((T + 1, m.dx))
    y = np.zeros((T, m.dy))
    lib().or_simulate(m.ref, C.c_uint64(seed), T, _d(xt), _d(y))
    return xt, y


def kalman_ou(m: Model, y):
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(-1))
    mean_ = np.zeros(y.size)
    var_ = np.zeros(y.size)
    ll = lib().or_kalman_ou(m.ref, y.size, _d(y), _d(mean_), _d(var_))
    return mean_, var_, ll


# ---------------------------------------------------------------------------
# Learned proposal (drift correction u_theta with exact increment-ratio
# weights; see pf_oracle.h).  Parameter vectors are float64 in the order
# W1[64][in], b1[64], W2[64][64], b2[64], W3[out][64], b3[out].

HIDDEN = 64


def mlp_nparams(in_dim, out_dim) -> int:
    return int(lib().or_mlp_nparams(in_dim, out_dim))


def mlp_unpack(p, in_dim, out_dim):
    """Views (W1, b1, W2, b2, W3, b3) of a flat parameter vector."""
    H = HIDDEN
    sizes = [H * in_dim, H, H * H, H, out_dim * H, out_dim]
    shapes = [(H, in_dim), (H,), (H, H), (H,), (out_dim, H), (out_dim,)]
    out, o = [], 0
    for n, sh in zip(sizes, shapes):
        out.append(p[o:o + n].reshape(sh))
        o += n
    return out


def bf16(x) -> np.ndarray:
    f = lib().or_bf16
    return np.vectorize(lambda v: f(float(v)), otypes=[np.float64])(np.asarray(x, np.float64))


def mlp_forward(p, x, out_dim, bf16_mode=False):
    """u_theta at the rows of x[B, in_dim]: returns (out[B, out_dim], h1, h2)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    B, in_dim = x.shape
    out = np.zeros((B, out_dim))
    h1 = np.zeros((B, HIDDEN))
    h2 = np.zeros((B, HIDDEN))
    for r in range(B):
        lib().or_mlp_forward(in_dim, out_dim, _d(p), _d(x[r]), _d(h1[r]), _d(h2[r]), _d(out[r]),
                             int(bf16_mode))
    return out, h1, h2


def mlp_backward(p, x, dout) -> np.ndarray:
    """d(dout . u_theta(x)) / dp for one row."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    dout = np.ascontiguousarray(dout, dtype=np.float64)
    g = np.zeros_like(p)
    lib().or_mlp_backward(x.size, dout.size, _d(p), _d(x), _d(dout), _d(g))
    return g


def mlp_loss_grad(p, X, T):
    """Mean squared regression loss over the rows of X onto T and its gradient."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.zeros_like(p)
    loss = lib().or_mlp_loss_grad(X.shape[1], T.shape[1], _d(p), X.shape[0], _d(X), _d(T), _d(g))
    return loss, g


def nearest_obs(m: Model) -> np.ndarray:
    out = np.zeros(m.J * m.J, np.int32)
    lib().or_nearest_obs(m.ref, _i32(out))
    return out


FHN_FEATURES = 22


def fhn_features(m: Model, x, y, k, nodes=None) -> np.ndarray:
    """features[len(nodes), 22] of one FH-N state at step k of the interval."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    near = nearest_obs(m)
    nodes = range(m.J * m.J) if nodes is None else nodes
    out = np.zeros((len(nodes), FHN_FEATURES))
    for r, n in enumerate(nodes):
        lib().or_fhn_features(m.ref, _d(x), _d(y), _i32(near), k, int(n), _d(out[r]))
    return out


def ou_features(m: Model, x, y, k) -> np.ndarray:
    f = np.zeros(3)
    lib().or_ou_features(m.ref, _d(np.array([x], np.float64)), _d(np.array([y], np.float64)), k,
                         _d(f))
    return f


def propagate_learned(m: Model, p, seed, filt, t, X, y, bf16_mode=True):
    """Interval t under the learned proposal: returns (X', dlw[N])."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    p = np.ascontiguousarray(p, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    dlw = np.zeros(X.shape[0])
    lib().or_propagate_learned(m.ref, _d(p), C.c_uint64(seed), filt, X.shape[0], t, _d(X),
                               _d(y), _d(dlw), int(bf16_mode))
    return X, dlw


def propagate_learned_particle(m: Model, p, seed, filt, index, t, x, y, bf16_mode=True):
    """Interval t of one particle (Philox counter word 0 = index) under the
    learned proposal: returns (x', its log increment-density ratio)."""
    x = np.array(x, dtype=np.float64, copy=True)
    p = np.ascontiguousarray(p, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    r = lib().or_propagate_learned_particle(m.ref, _d(p), C.c_uint64(seed), filt, index, t,
                                            _d(x), _d(y), int(bf16_mode))
    return x, float(r)


def filter_interval_learned(m: Model, p, seed, filt, t, X, y, logZ=0.0, bf16_mode=True):
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    p = np.ascontiguousarray(p, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    N = X.shape[0]
    lz = C.c_double(logZ)
    lw = np.zeros(N)
    A = np.zeros(N, np.int32)
    mp = np.zeros(m.dx)
    mw = np.zeros(m.dx)
    ess = C.c_double()
    deg = lib().or_filter_interval_learned(m.ref, _d(p), C.c_uint64(seed), filt, N, t, _d(X),
                                           _d(y), C.byref(lz), _d(lw), _i32(A), _d(mp), _d(mw),
                                           C.byref(ess), int(bf16_mode))
    return dict(X=X, lw=lw, A=A, mean_post=mp, mean_w=mw, logZ=lz.value, ess=ess.value,
                degenerate=bool(deg))


def run_ensemble_learned(m: Model, p, seed, M, N, y, bf16_mode=True):
    y = np.ascontiguousarray(y, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    T = y.shape[0]
    est = np.zeros((T, m.dx))
    est_w = np.zeros((T, m.dx))
    logZ = np.zeros(M)
    ess = np.zeros(T)
    lib().or_run_ensemble_learned(m.ref, _d(p), C.c_uint64(seed), M, N, T, _d(y), _d(est),
                                  _d(est_w), _d(logZ), _d(ess), int(bf16_mode))
    return est, est_w, logZ, ess


def ou_optimal_u(m: Model, x, y, k) -> float:
    return float(lib().or_ou_optimal_u(m.ref, float(x), float(y), int(k)))


# ---------------------------------------------------------------------------
# Training data of the learned proposal and Adam (definitions in pf_oracle.h)
TRAIN_RUN, TRAIN_TRAJ, TRAIN_BATCH = 0xFFFFFFFE, 0xFFFFFFFD, 0xFFFFFFFC


def train_run(m: Model, seed, q, run_len) -> np.ndarray:
    out = np.zeros((run_len, m.dx))
    lib().or_train_run(m.ref, C.c_uint64(seed), q, run_len, _d(out))
    return out


def train_trajectory(m: Model, seed, r, x0):
    """(states before each step [S, dx], y [dy], noise [S, dx])."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    traj = np.zeros((m.S, m.dx))
    y = np.zeros(m.dy)
    z = np.zeros((m.S, m.dx))
    lib().or_train_trajectory(m.ref, C.c_uint64(seed), r, _d(x0), _d(traj), _d(y), _d(z))
    return traj, y, z


def train_tile(m: Model, seed, n_traj, step, b):
    r, k, n0 = C.c_int(), C.c_int(), C.c_int()
    lib().or_train_tile(m.ref, C.c_uint64(seed), n_traj, step, b, C.byref(r), C.byref(k),
                        C.byref(n0))
    return r.value, k.value, n0.value


def adam_step(p, g, mo, ve, lr, beta1, beta2, eps, t):
    """In place on float64 arrays p, mo, ve."""
    lib().or_adam_step(p.size, _d(p), _d(np.ascontiguousarray(g, dtype=np.float64)), _d(mo),
                       _d(ve), lr, beta1, beta2, eps, t)
