"""MI355X-native independent-ensemble particle filter (arXiv 1407.8071).

Thin ctypes binding over ``libpf.so`` (the C ABI of ``include/pf.h``).  This
module only marshals arguments: every step of the filter runs in the HIP
kernels of the shared library.  PyTorch provides device memory (the
workspace and all tensors) and the current HIP stream.  If ``libpf.so`` is
missing the import of the binding fails loudly; there is no CPU fallback.

Model dictionaries (see ``PFModel``): kind ('ou1d' | 'lorenz63' | 'fhn'), dx,
J, S, h, params, noise_sd, obs_idx, obs_var, prior_mean, prior_sd.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpf.so")

KIND = {"ou1d": 0, "lorenz63": 1, "fhn": 2, "fhn_paper": 3}
OPT_PLAIN, OPT_FUSED, OPT_GRAPH = 0, 1, 2
STAGE_PROPAGATE, STAGE_WEIGHT, STAGE_RESAMPLE, STAGE_GATHER, STAGE_ESTIMATE = 1, 2, 4, 8, 16
STAGE_ALL = 31
ENS_LEARNED = 1
ENS_AUXILIARY = 2


class PFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pf status {status}: {msg}")
        self.status = status


class _ModelDesc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("state_dim", C.c_int32), ("grid_j", C.c_int32),
        ("steps_per_obs", C.c_int32), ("h", C.c_double), ("params", C.c_double * 4),
        ("noise_sd", C.c_double * 2), ("obs_dim", C.c_int32),
        ("h_obs_index", C.POINTER(C.c_int32)), ("obs_var", C.c_double),
        ("h_prior_mean", C.POINTER(C.c_double)), ("h_prior_sd", C.POINTER(C.c_double)),
        ("params_ext", C.c_double * 8),
    ]


class _Tuning(C.Structure):
    _fields_ = [("vec_single_kernel", C.c_int32), ("prop_tile", C.c_int32),
                ("resample_bd_min", C.c_int32), ("grid_blocks_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class _TrainDesc(C.Structure):
    _fields_ = [("n_runs", C.c_int32), ("run_len", C.c_int32), ("batch_tiles", C.c_int32),
                ("reserved", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64)]


class _EnsDesc(C.Structure):
    _fields_ = [("model", C.c_int32), ("M", C.c_int32), ("N", C.c_int32),
                ("flags", C.c_uint32), ("seed", C.c_uint64), ("scheme", C.c_int32),
                ("reserved", C.c_int32), ("ess_threshold", C.c_double)]


# resampling schemes of pf_ensemble_desc.scheme
RESAMPLE = {"multinomial": 0, "systematic": 1, "stratified": 2, "residual": 3}


_lib = None
_VP = C.c_void_p


def lib():
    """Load libpf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1407_8071_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    i32, u32, u64, i64 = C.c_int32, C.c_uint32, C.c_uint64, C.c_int64
    MD, ED = C.POINTER(_ModelDesc), C.POINTER(_EnsDesc)
    sigs = {
        "pf_workspace_bytes": [MD, i32, ED, i32, u32, C.POINTER(C.c_size_t)],
        "pf_init": [MD, i32, ED, i32, u32, _VP, C.c_size_t, _VP, C.POINTER(_VP)],
        "pf_step": [_VP, _VP, _VP],
        "pf_run_stages": [_VP, u32, _VP, _VP],
        "pf_estimate": [_VP, _VP, _VP, _VP, _VP, _VP],
        "pf_set_particles": [_VP, i32, _VP, _VP],
        "pf_get_particles": [_VP, i32, _VP, _VP],
        "pf_get_predicted": [_VP, i32, _VP, _VP],
        "pf_set_predicted": [_VP, i32, _VP, _VP],
        "pf_get_logweights": [_VP, i32, _VP, _VP],
        "pf_set_logweights": [_VP, i32, _VP, _VP],
        "pf_get_carried_logweights": [_VP, i32, _VP, _VP],
        "pf_set_carried_logweights": [_VP, i32, _VP, _VP],
        "pf_get_ancestors": [_VP, i32, _VP, _VP],
        "pf_get_filter_stats": [_VP, i32, _VP, _VP],
        "pf_set_interval": [_VP, i32],
        "pf_set_observations": [_VP, _VP, i32],
        "pf_get_interval": [_VP, C.POINTER(i32)],
        "pf_simulate": [_VP, i32, u64, i32, _VP, _VP, _VP],
        "pf_philox_stream": [u64, u32, u32, u32, i64, _VP, _VP, _VP],
        "pf_sync": [_VP],
        "pf_set_profiling": [_VP, i32],
        "pf_read_profile": [_VP, C.POINTER(C.c_double), C.POINTER(i64)],
        "pf_proposal_set": [_VP, i32, _VP, i64, _VP],
        "pf_get_tuning": [_VP, C.POINTER(_Tuning)],
        "pf_set_tuning": [_VP, C.POINTER(_Tuning), _VP],
        "pf_autotune": [_VP, _VP, i32, _VP, C.POINTER(_Tuning)],
        "pf_mlp_forward": [_VP, i32, i32, _VP, i64, _VP, _VP],
        "pf_mlp_grad_work_bytes": [i32, i32, i64, C.POINTER(C.c_size_t)],
        "pf_mlp_loss_grad": [_VP, i32, i32, _VP, _VP, i64, _VP, _VP, _VP, C.c_size_t, _VP],
        "pf_mlp_loss_grad_noalloc": [_VP, i32, i32, _VP, _VP, i64, _VP, _VP, _VP],
        "pf_adam_step": [_VP, _VP, _VP, _VP, i64, C.c_double, C.c_double, C.c_double,
                         C.c_double, i32, _VP],
        "pf_train_workspace_bytes": [MD, C.POINTER(_TrainDesc), C.POINTER(C.c_size_t)],
        "pf_train_data": [MD, C.POINTER(_TrainDesc), _VP, C.c_size_t, _VP],
        "pf_train_buffers": [MD, C.POINTER(_TrainDesc), _VP, C.POINTER(_VP), C.POINTER(_VP),
                             C.POINTER(_VP)],
        "pf_train_steps": [MD, C.POINTER(_TrainDesc), _VP, C.c_size_t, _VP, i32, i32, _VP, _VP],
        "pf_train_grad": [MD, C.POINTER(_TrainDesc), _VP, C.c_size_t, _VP, i32, _VP, _VP, _VP],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.pf_mlp_nparams.argtypes = [i32, i32]
    L.pf_mlp_nparams.restype = i32
    L.pf_destroy.argtypes = [_VP]
    L.pf_destroy.restype = None
    L.pf_status_str.argtypes = [C.c_int]
    L.pf_status_str.restype = C.c_char_p
    L.pf_last_error.argtypes = []
    L.pf_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise PFError(status, lib().pf_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class PFModel:
    """Marshals a model dictionary into a pf_model_desc (keeps arrays alive)."""

    def __init__(self, spec: dict):
        self.spec = dict(spec)
        self.dx = int(spec["dx"])
        self.obs_idx = np.ascontiguousarray(spec["obs_idx"], dtype=np.int32)
        self.dy = int(self.obs_idx.size)
        self.prior_mean = np.ascontiguousarray(spec["prior_mean"], dtype=np.float64)
        self.prior_sd = np.ascontiguousarray(spec["prior_sd"], dtype=np.float64)
        p = list(spec["params"]) + [0.0] * (4 - len(spec["params"]))
        sd = list(spec["noise_sd"]) + [0.0] * (2 - len(spec["noise_sd"]))
        self.desc = _ModelDesc(
            KIND[spec["kind"]], self.dx, int(spec.get("J", 0)), int(spec["S"]),
            float(spec["h"]), (C.c_double * 4)(*p), (C.c_double * 2)(*sd), self.dy,
            self.obs_idx.ctypes.data_as(C.POINTER(C.c_int32)), float(spec["obs_var"]),
            self.prior_mean.ctypes.data_as(C.POINTER(C.c_double)),
            self.prior_sd.ctypes.data_as(C.POINTER(C.c_double)),
            (C.c_double * 8)(*(list(spec.get("params_ext", ())) +
                               [0.0] * (8 - len(spec.get("params_ext", ()))))))


# Contexts still open.  They are closed by an exit handler, which runs
# before the interpreter tears its modules down and before the HIP runtime's
# own exit-time teardown, so that no context is destroyed from a finaliser
# after the runtime has gone.
_LIVE: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    for f in list(_LIVE):
        try:
            f.close()
        except Exception:
            pass


class ParticleFilter:
    """A context of one or more ensembles of independent bootstrap filters.

    ``ensembles`` is a list of (model_index, M, N, seed[, flags[, scheme[,
    ess_threshold]]]) with flags 0 or ENS_LEARNED, scheme a name of RESAMPLE
    or its number, ess_threshold 0 (resample every interval) or in (0, 1].  ``fused``
    selects the persistent fused interval kernel instead of one kernel per
    step.
    """

    def __init__(self, models, ensembles, fused: bool = False, graph: bool = False, stream=None):
        import torch
        self.models = [m if isinstance(m, PFModel) else PFModel(m) for m in models]
        self.ens = [tuple(e) for e in ensembles]
        nm, ne = len(self.models), len(self.ens)
        self._md = (_ModelDesc * nm)(*[m.desc for m in self.models])
        def desc(e):
            mi, M, N, seed = e[:4]
            flags = e[4] if len(e) > 4 else 0
            scheme = e[5] if len(e) > 5 else 0
            scheme = RESAMPLE[scheme] if isinstance(scheme, str) else int(scheme)
            ess = float(e[6]) if len(e) > 6 else 0.0
            return _EnsDesc(int(mi), int(M), int(N), int(flags), int(seed), scheme, 0, ess)
        self._ed = (_EnsDesc * ne)(*[desc(e) for e in self.ens])
        self.options = (OPT_FUSED if fused or graph else OPT_PLAIN) | (OPT_GRAPH if graph else 0)
        nbytes = C.c_size_t()
        _check(lib().pf_workspace_bytes(self._md, nm, self._ed, ne, self.options,
                                        C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self.workspace = torch.empty(max(1, nbytes.value) + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self._ws = C.c_void_p((base + 255) // 256 * 256)
        ctx = C.c_void_p()
        _check(lib().pf_init(self._md, nm, self._ed, ne, self.options, self._ws,
                             nbytes.value, _stream(stream), C.byref(ctx)))
        self._ctx = ctx
        _LIVE.add(self)

    def close(self):
        """Release the context (waits for its queued work); idempotent."""
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            lib().pf_destroy(ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- shapes ------------------------------------------------------------
    def dims(self, e: int):
        mi, M, N = self.ens[e][:3]
        return self.models[mi], M, N

    def particle_shape(self, e: int):
        m, M, N = self.dims(e)
        if m.spec["kind"] in ("fhn", "fhn_paper"):
            return (M, N, m.dx)
        return (M, m.dx, N)

    # ---- the filter --------------------------------------------------------
    def step(self, y=None, stream=None):
        """One interval; y=None reads the record staged by set_observations."""
        _check(lib().pf_step(self._ctx, _ptr(y), _stream(stream)))

    def set_observations(self, y_all):
        """Stage y_all [T, sum obs_dim] (float32, on the device; kept referenced)."""
        import torch
        assert y_all.dtype == torch.float32 and y_all.is_cuda and y_all.is_contiguous()
        self._y_all = y_all
        _check(lib().pf_set_observations(self._ctx, _ptr(y_all), int(y_all.shape[0])))

    def run_stages(self, stages: int, y=None, stream=None):
        _check(lib().pf_run_stages(self._ctx, stages, _ptr(y), _stream(stream)))

    def estimate(self, stream=None):
        import torch
        dx = sum(self.models[mi].dx for (mi, *_) in self.ens)
        nM = sum(M for (_, M, *_) in self.ens)
        nF = sum(M * self.models[mi].dx for (mi, M, *_) in self.ens)
        mean = torch.empty(dx, dtype=torch.float64, device="cuda")
        mean_w = torch.empty(dx, dtype=torch.float64, device="cuda")
        logZ = torch.empty(nM, dtype=torch.float64, device="cuda")
        fmean = torch.empty(nF, dtype=torch.float64, device="cuda")
        _check(lib().pf_estimate(self._ctx, _ptr(mean), _ptr(mean_w), _ptr(logZ), _ptr(fmean),
                                 _stream(stream)))
        return mean, mean_w, logZ, fmean

    # ---- hooks -------------------------------------------------------------
    def set_particles(self, e: int, x, stream=None):
        import torch
        assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
        assert tuple(x.shape) == self.particle_shape(e)
        _check(lib().pf_set_particles(self._ctx, e, _ptr(x), _stream(stream)))

    def _get(self, fn, e, shape, dtype, stream):
        import torch
        out = torch.empty(shape, dtype=dtype, device="cuda")
        _check(fn(self._ctx, e, _ptr(out), _stream(stream)))
        return out

    def get_particles(self, e: int, stream=None):
        import torch
        return self._get(lib().pf_get_particles, e, self.particle_shape(e), torch.float32, stream)

    def get_predicted(self, e: int, stream=None):
        import torch
        return self._get(lib().pf_get_predicted, e, self.particle_shape(e), torch.float32, stream)

    def set_predicted(self, e: int, x, stream=None):
        import torch
        assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
        assert tuple(x.shape) == self.particle_shape(e)
        _check(lib().pf_set_predicted(self._ctx, e, _ptr(x), _stream(stream)))

    def get_logweights(self, e: int, stream=None):
        import torch
        _, M, N = self.dims(e)
        return self._get(lib().pf_get_logweights, e, (M, N), torch.float32, stream)

    def set_logweights(self, e: int, lw, stream=None):
        import torch
        _, M, N = self.dims(e)
        assert lw.dtype == torch.float32 and lw.is_cuda and tuple(lw.shape) == (M, N)
        _check(lib().pf_set_logweights(self._ctx, e, _ptr(lw.contiguous()), _stream(stream)))

    def get_carried_logweights(self, e: int, stream=None):
        import torch
        _, M, N = self.dims(e)
        return self._get(lib().pf_get_carried_logweights, e, (M, N), torch.float32, stream)

    def set_carried_logweights(self, e: int, lwc, stream=None):
        import torch
        _, M, N = self.dims(e)
        assert lwc.dtype == torch.float32 and lwc.is_cuda and tuple(lwc.shape) == (M, N)
        _check(lib().pf_set_carried_logweights(self._ctx, e, _ptr(lwc.contiguous()),
                                               _stream(stream)))

    def get_ancestors(self, e: int, stream=None):
        import torch
        _, M, N = self.dims(e)
        return self._get(lib().pf_get_ancestors, e, (M, N), torch.int32, stream)

    def get_filter_stats(self, e: int, stream=None):
        import torch
        _, M, _ = self.dims(e)
        return self._get(lib().pf_get_filter_stats, e, (M, 4), torch.float64, stream)

    def set_interval(self, t: int):
        _check(lib().pf_set_interval(self._ctx, t))

    def interval(self) -> int:
        t = C.c_int32()
        _check(lib().pf_get_interval(self._ctx, C.byref(t)))
        return t.value

    def simulate(self, e: int, seed: int, T: int, stream=None):
        import torch
        m, _, _ = self.dims(e)
        xt = torch.empty((T + 1, m.dx), dtype=torch.float32, device="cuda")
        y = torch.empty((T, m.dy), dtype=torch.float32, device="cuda")
        _check(lib().pf_simulate(self._ctx, e, seed, T, _ptr(xt), _ptr(y), _stream(stream)))
        return xt, y

    # ---- launch-shape tuning -------------------------------------------------
    def tuning(self) -> dict:
        u = _Tuning()
        _check(lib().pf_get_tuning(self._ctx, C.byref(u)))
        return u.as_dict()

    def set_tuning(self, tuning: dict, stream=None):
        u = _Tuning(**{k: int(v) for k, v in tuning.items()})
        _check(lib().pf_set_tuning(self._ctx, C.byref(u), _stream(stream)))

    def autotune(self, y, reps: int = 5, stream=None) -> dict:
        """Time candidate launch plans on the device with observations y (one
        interval), keep the fastest; the filters restart from their prior."""
        u = _Tuning()
        _check(lib().pf_autotune(self._ctx, _ptr(y), reps, _stream(stream), C.byref(u)))
        return u.as_dict()

    def signature(self) -> str:
        """Batch shape that a tuning depends on: models and (M, N, flags)."""
        import hashlib
        parts = []
        for m in self.models:
            sp = m.spec
            parts.append(f"{sp['kind']}:{m.dx}:{sp.get('J', 0)}:{sp['S']}")
        parts += [f"{e[0]}:{e[1]}:{e[2]}:{e[4] if len(e) > 4 else 0}" for e in self.ens]
        return hashlib.sha1("|".join(parts).encode()).hexdigest()

    def autotune_cached(self, y, cache_path: str, reps: int = 5, stream=None) -> dict:
        """The tuning stored for this batch shape and device in the JSON file
        `cache_path`, else the autotuner's choice (then stored)."""
        import json
        import torch
        key = f"{torch.cuda.get_device_name()}|{self.signature()}"
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        if key in cache:
            self.set_tuning(cache[key], stream)
            return cache[key]
        t = self.autotune(y, reps, stream)
        cache[key] = t
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
        return t

    def set_proposal(self, e: int, params, stream=None):
        """Network of learned ensemble e (float32 device tensor, flat)."""
        _check(lib().pf_proposal_set(self._ctx, e, _ptr(params), params.numel(), _stream(stream)))

    def sync(self):
        _check(lib().pf_sync(self._ctx))

    def set_profiling(self, enable: bool):
        _check(lib().pf_set_profiling(self._ctx, 1 if enable else 0))

    def read_profile(self):
        """(summed milliseconds, launches) of the dominant kernel since the last read."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().pf_read_profile(self._ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def mlp_nparams(in_dim: int, out_dim: int) -> int:
    n = int(lib().pf_mlp_nparams(in_dim, out_dim))
    if n < 0:
        raise PFError(1, "in_dim must be in [1, 31] and out_dim in [1, 4]")
    return n


def mlp_forward(params, x, out_dim: int, stream=None):
    """u_theta over the rows of x [rows, in_dim] (float32 device tensors)."""
    import torch
    rows, in_dim = x.shape
    out = torch.empty((rows, out_dim), dtype=torch.float32, device="cuda")
    _check(lib().pf_mlp_forward(_ptr(params), in_dim, out_dim, _ptr(x), rows, _ptr(out),
                                _stream(stream)))
    return out


def mlp_loss_grad(params, x, target, stream=None):
    """(loss, grad) of the mean squared regression loss over the rows."""
    import torch
    rows, in_dim = x.shape
    out_dim = target.shape[1]
    n = C.c_size_t()
    _check(lib().pf_mlp_grad_work_bytes(in_dim, out_dim, rows, C.byref(n)))
    work = torch.empty(n.value // 4 + 1, dtype=torch.float32, device="cuda")
    grad = torch.empty(params.numel(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().pf_mlp_loss_grad(_ptr(params), in_dim, out_dim, _ptr(x), _ptr(target), rows,
                                  _ptr(grad), _ptr(loss), _ptr(work), n.value, _stream(stream)))
    return loss, grad


def mlp_loss_grad_noalloc(params, x, target, grad, loss, stream=None):
    """pf_mlp_loss_grad_noalloc into caller-owned grad and loss (float32
    device tensors): the library's static partial-gradient buffer instead of
    a work buffer, so the call allocates nothing."""
    rows, in_dim = x.shape
    out_dim = target.shape[1]
    _check(lib().pf_mlp_loss_grad_noalloc(_ptr(params), in_dim, out_dim, _ptr(x), _ptr(target),
                                          rows, _ptr(grad), _ptr(loss), _stream(stream)))


def adam_step(params, grad, m, v, lr, beta1, beta2, eps, t, stream=None):
    _check(lib().pf_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), lr,
                              beta1, beta2, eps, t, _stream(stream)))


class Trainer:
    """Training of an FH-N learned proposal on model-simulated paths."""

    def __init__(self, spec: dict, n_runs: int, run_len: int, batch_tiles: int, lr: float = 1e-3,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, seed: int = 1):
        import torch
        self.model = spec if isinstance(spec, PFModel) else PFModel(spec)
        self.desc = _TrainDesc(n_runs, run_len, batch_tiles, 0, lr, beta1, beta2, eps, seed)
        n = C.c_size_t()
        _check(lib().pf_train_workspace_bytes(C.byref(self.model.desc), C.byref(self.desc),
                                              C.byref(n)))
        self.nbytes = n.value
        self.work = torch.empty(n.value + 256, dtype=torch.uint8, device="cuda")
        self._ws = C.c_void_p((self.work.data_ptr() + 255) // 256 * 256)
        self.n_traj = n_runs * run_len
        self.step_count = 0

    def data(self, stream=None):
        _check(lib().pf_train_data(C.byref(self.model.desc), C.byref(self.desc), self._ws,
                                   self.nbytes, _stream(stream)))

    def buffers(self):
        """(start states, trajectories, observations) as device tensors (views)."""
        import torch
        ptrs = [C.c_void_p() for _ in range(3)]
        _check(lib().pf_train_buffers(C.byref(self.model.desc), C.byref(self.desc), self._ws,
                                      *[C.byref(p) for p in ptrs]))
        m, S = self.model, int(self.model.spec["S"])
        base = self.work.data_ptr()
        def view(p, shape):
            off = p.value - base
            n = int(np.prod(shape))
            return self.work[off:off + 4 * n].view(torch.float32).view(*shape)
        return (view(ptrs[0], (self.n_traj, m.dx)), view(ptrs[1], (self.n_traj, S, m.dx)),
                view(ptrs[2], (self.n_traj, m.dy)))

    def grad(self, params, step: int, stream=None):
        """(loss, gradient) of the minibatch of Adam step `step`, no update."""
        import torch
        g = torch.empty(params.numel(), dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().pf_train_grad(C.byref(self.model.desc), C.byref(self.desc), self._ws,
                                   self.nbytes, _ptr(params), step, _ptr(g), _ptr(loss),
                                   _stream(stream)))
        return loss, g

    def steps(self, params, n_steps: int, stream=None):
        """Run n_steps Adam steps on params (float32 device tensor); returns the losses."""
        import torch
        loss = torch.empty(max(1, n_steps), dtype=torch.float32, device="cuda")
        _check(lib().pf_train_steps(C.byref(self.model.desc), C.byref(self.desc), self._ws,
                                    self.nbytes, _ptr(params), self.step_count + 1, n_steps,
                                    _ptr(loss), _stream(stream)))
        self.step_count += n_steps
        return loss[:n_steps]


def philox_stream(seed: int, c1: int, c2: int, c3: int, n: int, stream=None):
    """Philox words and Box-Muller normals from the device generator."""
    import torch
    bits = torch.empty(n, dtype=torch.int32, device="cuda")
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().pf_philox_stream(seed, c1, c2, c3, n, _ptr(bits), _ptr(z), _stream(stream)))
    return bits, z
